#!/usr/bin/env python3
"""Throughput of Frobenius inversion on one MI355X.

Workload (default): one n = 4096 FP64 general complex matrix M = A + iB with
A, B iid N(0, 1) (seed 0).  A step is one Frobenius inversion of M through the
C ABI (Algorithm 5: LU of A, Y = A^{-1} B, C = A + B Y, C^{-1}, -Y C^{-1}),
inputs resident in HBM, ending with the call's own synchronization.  The
value is inversions per second on this one GPU.

Also measured (outside the timed steps, same protocol): the HPD path
(Algorithm 7) on M = Z Z^H + n I, and the complex-arithmetic baselines
(Algorithms 4 and 8, both as printed and in LAPACK getri/potri form); the
mixed-precision variant (FP32 / BF16 matrix-core operands plus Newton-Schulz
refinement with an FP64 residual) on the same matrices; the batched line
(2048 matrices, orders uniform in [16, 512], half general and half HPD, one
persistent launch, FP64 and FP32) beside a per-matrix complex-LU loop on a
sample of it; and the adjoint (256 HPD matrices of order 256, dM = -X^H G X^H
by three-multiplication complex products, FP32 and FP64).  The dominant kernel (the n x n x n FP64 matrix-core
GEMM) is timed with HIP events on the library's stream during the timed steps
and reported against the FP64 matrix peak.  The CPU baseline is the FP64
oracle of the test suite timed on this host on a smaller matrix of the same
recipe and scaled by n^3.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip HPD and baseline measurements")
    ap.add_argument("--cpu-n", type=int, default=1536)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _events_ms(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(fi, inputs, h, torch, np, log):
    """2048 matrices, n ~ U{16..512} (seed 4), kind = i mod 2: one persistent launch."""
    log("[bench] batched: generating 2048 matrices")
    ns, kinds, mats = inputs.batch(count=2048, seed=4)
    flops = float(np.sum(np.where(kinds == 0, 26.0 / 3.0, 19.0 / 3.0) * ns.astype(np.float64) ** 3))
    out = {}
    fi.frob_batched_tune(h, fi.FROB_PREC_F64)
    fi.frob_batched_tune(h, fi.FROB_PREC_F32)
    for dt, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
        As = [torch.from_numpy(A).to(dt).cuda() for A, _ in mats]
        Bs = [torch.from_numpy(B).to(dt).cuda() for _, B in mats]
        plan = fi.BatchedPlan(As, Bs, kinds)
        ms = _events_ms(torch, lambda: plan.launch(h))
        bad = int((plan.info_dev != 0).sum())
        out[f"batched_{tag}"] = {"ms": ms, "inversions_per_s": 2048 / (ms * 1e-3), "alg_tflops": flops / ms / 1e9,
                                 "nonzero_info": bad}
        log(f"[bench] batched {tag}: {ms:.2f} ms")
        del As, Bs, plan
    # baseline: per-matrix complex-LU / complex-Cholesky loop on a sample, scaled to the batch
    idx = np.arange(0, 2048, 32)
    Ms = [(torch.from_numpy(mats[i][0]).cuda(), torch.from_numpy(mats[i][1]).cuda()) for i in idx]

    def loop():
        for (a, b), i in zip(Ms, idx):
            (fi.frob_cinv_lu if kinds[i] == 0 else fi.frob_cinv_chol)(h, a, b)
    ms = _events_ms(torch, loop, reps=1)
    out["per_matrix_complex_loop_sampled"] = {"ms_sample": ms, "sample": len(idx),
                                              "ms_scaled_to_2048": ms * 2048 / len(idx)}
    return out


def bench_adjoint(fi, inputs, h, torch, np, log):
    """256 HPD matrices of order 256 (seed 5): X by the batched FP32 inversion,
    then dM = -X^H W^H X^H."""
    log("[bench] adjoint: generating 256 HPD matrices")
    mats, ws = inputs.adjoint_batch(count=256, n=256, seed=5)
    n, b = 256, 256
    out = {}
    for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
        As = [torch.from_numpy(A).to(dt).cuda() for A, _ in mats]
        Bs = [torch.from_numpy(B).to(dt).cuda() for _, B in mats]
        plan = fi.BatchedPlan(As, Bs, [1] * b)
        fwd_ms = _events_ms(torch, lambda: plan.launch(h))
        Xr = torch.stack(plan.Xr).contiguous()
        Xi = torch.stack(plan.Xi).contiguous()
        Gr = torch.from_numpy(np.stack([w[0].T for w in ws])).to(dt).cuda().contiguous()
        Gi = torch.from_numpy(np.stack([-w[1].T for w in ws])).to(dt).cuda().contiguous()
        dMr, dMi = torch.empty_like(Xr), torch.empty_like(Xr)
        ms = _events_ms(torch, lambda: fi.frob_inv_adjoint(h, Xr, Xi, Gr, Gi, dMr, dMi))
        out[f"adjoint_{tag}"] = {"forward_batched_ms": fwd_ms, "backward_ms": ms,
                                 "backward_tflops_3m": 12.0 * b * n ** 3 / ms / 1e9}
        log(f"[bench] adjoint {tag}: forward {fwd_ms:.2f} ms, backward {ms:.3f} ms")
        del As, Bs, plan, Xr, Xi, Gr, Gi, dMr, dMi
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (multi-GPU sharding of the "
              "inversion is not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": nbytes, "copies": 3}), flush=True)
        return

    import paper_2208_01239_amd as fi
    from paper_2208_01239_amd import inputs

    n, K, W = args.n, args.steps, args.warmup
    torch.cuda.set_device(0)
    log(f"[bench] generating inputs n={n}")
    A, B = inputs.general(n, 0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Xr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    Xi = torch.empty_like(Xr)
    h = fi.Handle(0)

    def step():
        fi.frob_inv_general(h, dA, dB, Xr, Xi)

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    log(f"[bench] frobenius general: warmup {W}, steps {K}")
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / K
    launches, gemm_ms, gemm_flops = h.profile_read(0)
    h.profile(False)
    log(f"[bench] frobenius general: {t_step * 1e3:.3f} ms/step")

    # accuracy on sampled columns: backward error ||M x_j - e_j|| / (||M|| ||x_j||)
    rng = np.random.default_rng(123)
    cols = np.sort(rng.choice(n, size=min(8, n), replace=False))
    xr = Xr[:, cols].cpu().numpy()
    xi = Xi[:, cols].cpu().numpy()
    E = np.zeros((n, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    Rr = A @ xr - B @ xi - E
    Ri = A @ xi + B @ xr
    normM = np.linalg.norm(A, 2) if n <= 2048 else np.sqrt(np.sum(A * A) + np.sum(B * B))
    berr = float(np.sqrt(np.sum(Rr ** 2 + Ri ** 2)) / (normM * np.sqrt(np.sum(xr ** 2 + xi ** 2))))
    gold = os.path.join(ROOT, "tests", "golden", f"n{n}_general_samples.npz")
    relf_samples = None
    if os.path.exists(gold):
        g = np.load(gold, allow_pickle=False)
        gc = g["cols"]
        gr, gi = Xr[:, gc].cpu().numpy(), Xi[:, gc].cpu().numpy()
        relf_samples = float(np.sqrt(np.sum((gr - g["xr"]) ** 2 + (gi - g["xi"]) ** 2) /
                                     np.sum(g["xr"] ** 2 + g["xi"] ** 2)))

    extra = {}
    if not args.no_extra:
        log("[bench] frobenius HPD")
        Ah, Bh = inputs.hpd(n, 1)
        dAh, dBh = torch.from_numpy(Ah).cuda(), torch.from_numpy(Bh).cuda()
        t_hpd = timed(lambda: fi.frob_inv_hpd(h, dAh, dBh, Xr, Xi), max(2, K // 2), 1)
        extra["hpd_ms"] = t_hpd * 1e3
        extra["hpd_inversions_per_s"] = 1.0 / t_hpd
        extra["hpd_eff_tflops_4n3"] = 4.0 * n ** 3 / t_hpd / 1e12
        for name, fn, Mr, Mi in (("cinv_lu", fi.frob_cinv_lu, dA, dB), ("cinv_chol", fi.frob_cinv_chol, dAh, dBh)):
            for form in (1, 0):
                try:
                    t = timed(lambda: fn(h, Mr, Mi, Xr, Xi, form=form), max(2, K // 2), 1)
                    extra[f"{name}_form{form}_ms"] = t * 1e3
                except fi.FrobError as e:
                    extra[f"{name}_form{form}_ms"] = None
                    log(f"[bench] {name} form {form} unavailable: {e}")
        # mixed precision + Newton-Schulz (same general and HPD matrices)
        for tag, fn, Ma, Mb in (("mp_general", fi.frob_inv_general, dA, dB), ("mp_hpd", fi.frob_inv_hpd, dAh, dBh)):
            for pname, prec in (("f32", fi.FROB_PREC_F32), ("bf16", fi.FROB_PREC_BF16)):
                key = f"{tag}_{pname}"
                log(f"[bench] {key}")
                try:
                    res = {}

                    def run_mp():
                        res.update(fn(h, Ma, Mb, Xr, Xi, prec=prec, refine=8)[2])
                    t = timed(run_mp, 2, 1)
                    entry = {"ms": t * 1e3, "refine_steps": res["refine_steps"], "resid0": res["resid0"],
                             "resid": res["resid"]}
                    if tag == "mp_general" and os.path.exists(gold):
                        g = np.load(gold, allow_pickle=False)
                        gc = g["cols"]
                        gr, gi = Xr[:, gc].cpu().numpy(), Xi[:, gc].cpu().numpy()
                        entry["relF_vs_oracle_sampled_cols"] = float(np.sqrt(
                            np.sum((gr - g["xr"]) ** 2 + (gi - g["xi"]) ** 2) / np.sum(g["xr"] ** 2 + g["xi"] ** 2)))
                    extra[key] = entry
                except fi.FrobError as e:
                    extra[key] = {"status": str(e)}
        del dAh, dBh
        extra.update(bench_batched(fi, inputs, h, torch, np, log))
        extra.update(bench_adjoint(fi, inputs, h, torch, np, log))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = min(args.cpu_n, n)
        Ac, Bc = inputs.general(m, 0)
        log(f"[bench] cpu baseline: oracle Algorithm 5 at n={m}, {oracle.num_threads()} threads")
        tc0 = time.perf_counter()
        oracle.frob_lu(Ac, Bc)
        tc = time.perf_counter() - tc0
        scaled = tc * (n / m) ** 3
        cpu = {"value": 1.0 / scaled, "unit": "inversions/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"one n={m} general matrix of the same recipe (seed 0), Algorithm 5 in the FP64 oracle, "
                         f"{tc:.2f} s, scaled to n={n} by (n/{m})^3"}

    # HBM traffic of the dominant kernel from the committed rocprofv3 counter
    # summary, valid only while the kernel source is the one measured
    traffic = None
    tj = os.path.join(ROOT, "profiles", "gemm_f64_128x128_n4096_hbm_traffic.json")
    if n == 4096 and os.path.exists(tj):
        import hashlib
        with open(tj) as f:
            td = json.load(f)
        with open(os.path.join(ROOT, "paper_2208_01239_amd", "csrc", "gemm_f64.hip"), "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()
        if cur == td.get("gemm_f64_hip_sha256"):
            traffic = td["traffic_bytes_per_launch"]
    gemm_avg_ms = gemm_ms / launches if launches else None
    achieved = (gemm_flops / launches) / (gemm_avg_ms * 1e-3) / 1e12 if launches else None
    line = {
        "metric": "complex inversions/s & eff. TFLOP/s, Frobenius vs complex-LU at rel err <=1e-10",
        "value": 1.0 / t_step,
        "unit": "inversions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"frobenius_general_n{n}_fp64", "n": n, "generator": "A,B iid N(0,1) seed 0",
                   "batch": 1},
        "eff_tflops_8n3": 8.0 * n ** 3 / t_step / 1e12,
        "alg_tflops_26n3_3": (26.0 / 3.0) * n ** 3 / t_step / 1e12,
        "backward_error_sampled_cols": berr,
        "relF_vs_oracle_sampled_cols": relf_samples,
        "roofline": {"bound": "mfma", "kernel": "k_gemm_f64<128,128> (n x n x n products B*Y and -Y*C^-1)",
                     "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / FP64_MFMA_PEAK_TFLOPS) if achieved else None,
                     "avg_launch_ms": gemm_avg_ms, "launches": launches, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)"},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
