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
by three-multiplication complex products, FP32 and FP64); Frobenius against
complex-LU inversion at n = 8192 (same recipe, errors on the oracle's sampled
columns).  The roofline kernel is the look-ahead LUs' trailing-update GEMM
(FP64 matrix cores, on the library's second stream), timed with HIP events on
that stream during the timed steps; the n x n x n products are reported
beside it.  The CPU baseline is the FP64 oracle of the test suite timed on
this host on smaller matrices of the same recipe (all threads, and one
thread), scaled by n^3.  The JSON line on stdout carries the contract fields
and the headline comparison; every measurement is also written to
gpurun_out/bench_detail.json.

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
    ap.add_argument("--cpu-n", type=int, default=2048)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle once at the full order on all host threads (minutes)")
    ap.add_argument("--no-mp-large", action="store_true", help="skip the n = 8192 mixed-precision leg")
    ap.add_argument("--mp-n", type=int, default=8192)
    ap.add_argument("--no-large", action="store_true", help="skip the n = 8192 Frobenius / complex-LU comparison")
    ap.add_argument("--no-newton", action="store_true", help="skip the sign / polar / Sylvester legs")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 2048-matrix batched leg with the default panel widths (for kernel profiles)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint leg (256 HPD matrices of order 256; for kernel profiles)")
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


def bench_batched(fi, inputs, h, torch, np, log, tune=True, loop=True):
    """2048 matrices, n ~ U{16..512} (seed 4), kind = i mod 2: one persistent
    launch (panel widths autotuned first unless tune=False, then the default
    table), and a per-matrix complex-LU / complex-Cholesky loop on a sample."""
    log("[bench] batched: generating 2048 matrices")
    ns, kinds, mats = inputs.batch(count=2048, seed=4)
    flops = float(np.sum(np.where(kinds == 0, 26.0 / 3.0, 19.0 / 3.0) * ns.astype(np.float64) ** 3))
    out = {}
    if tune:
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
    if not loop:
        return out
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


def bench_newton(fi, inputs, h, torch, np, log, sizes=(2100, 4000)):
    """The paper's Section 5 workloads at its smallest and largest orders:
    matrix sign (n, tol 1e-3), polar decomposition (n, tol 1e-3) and the
    Sylvester equation (p = q = n / 2, tol 1e-1), each with every inverse by
    Frobenius inversion and by the complex-LU baseline (the comparison the
    paper makes), synthetic inputs of the paper's recipes; time per solve
    (one warm-up), Newton steps, and the relative max-norm error against the
    constructed solution."""
    out = {}

    def relmax(Xr, Xi, R):
        xr, xi = Xr.cpu().numpy(), Xi.cpu().numpy()
        return float(max(np.abs(xr - R.real).max(), np.abs(xi - R.imag).max()) / np.abs(R).max())

    def timed_call(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, r

    for n in sizes:
        log(f"[bench] newton workloads n={n}: generating")
        Xr, Xi, Sr, Si = inputs.sign_problem(n, seed=50)
        dXr, dXi = torch.from_numpy(Xr).cuda(), torch.from_numpy(Xi).cuda()
        X, Q, P = inputs.polar_problem(n, seed=52)
        dPr, dPi = torch.from_numpy(np.ascontiguousarray(X.real)).cuda(), torch.from_numpy(np.ascontiguousarray(X.imag)).cuda()
        p = n // 2
        A, B, C, Y = inputs.sylvester_problem(p, p, seed=51)
        dev = [torch.from_numpy(np.ascontiguousarray(f(M))).cuda() for M in (A, B, C) for f in (np.real, np.imag)]
        for tag, inv in (("frobenius", fi.FROB_NEWTON_FROBENIUS), ("complex_lu", fi.FROB_NEWTON_COMPLEX_LU)):
            ms, r = timed_call(lambda: fi.frob_sign(h, dXr, dXi, tol=1e-3, inverse=inv))
            out[f"newton_sign_n{n}_{tag}"] = {"ms": ms, "steps": r[2]["iterations"],
                                             "relmax_vs_closed_form": relmax(r[0], r[1], Sr + 1j * Si)}
            ms, r = timed_call(lambda: fi.frob_polar(h, dPr, dPi, tol=1e-3, inverse=inv))
            out[f"newton_polar_n{n}_{tag}"] = {"ms": ms, "steps": r[4]["iterations"],
                                              "relmax_Q": relmax(r[0], r[1], Q), "relmax_P": relmax(r[2], r[3], P)}
            ms, r = timed_call(lambda: fi.frob_sylvester(h, *dev, tol=1e-1, inverse=inv))
            out[f"newton_sylvester_p{p}_q{p}_{tag}"] = {"ms": ms, "steps": r[2]["iterations"],
                                                       "relmax_vs_constructed": relmax(r[0], r[1], Y)}
            for k in (f"newton_sign_n{n}_{tag}", f"newton_polar_n{n}_{tag}", f"newton_sylvester_p{p}_q{p}_{tag}"):
                log(f"[bench] {k}: {out[k]}")
        del dXr, dXi, dPr, dPi, dev
        torch.cuda.empty_cache()
    return out


def bench_mp_large(fi, inputs, h, torch, np, log, n):
    """Mixed precision at order n (8192): M = U diag(sigma) W (HPD:
    U diag(sigma) U^H) with kappa in {1e2, 1e4, 1e6}, U and W built from pair
    rotations on the device (inputs.spectrum_rotations; bit-identical to the
    host construction the oracle inverted).  For FP64, FP32 and BF16
    matrix-core operands, and FP64 with an FP32 Newton-Schulz correction: the
    error against the oracle's samples (tests/golden/n<n>_rot_*_band_samples
    .npz: one column per 64-column band, 256 rows) without refinement, and the
    time, step count, residual and error with up to eight Newton-Schulz steps
    (FP64 residual)."""
    import hashlib
    out = {}
    Xr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    Xi = torch.empty_like(Xr)
    for kind, fn, base in (("general", fi.frob_inv_general, 300), ("hpd", fi.frob_inv_hpd, 400)):
        for kexp in (2, 4, 6):
            log(f"[bench] mp n={n} {kind} kappa=1e{kexp}: generating")
            dA, dB = inputs.spectrum_rotations(n, 10.0 ** kexp, kind, seed=base + kexp, device="cuda")
            path = os.path.join(ROOT, "tests", "golden", f"n{n}_rot_{kind}_k1e{kexp}_band_samples.npz")
            g = np.load(path, allow_pickle=False) if os.path.exists(path) else None
            if g is not None:
                same = all(hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest() == str(g[k])
                           for t, k in ((dA, "sha_a"), (dB, "sha_b")))
                if not same:
                    log(f"[bench] mp {kind} 1e{kexp}: device input differs from the oracle's; errors not reported")
                    g = None
            if g is not None:
                rows = torch.from_numpy(g["rows"]).cuda()
                cols = torch.from_numpy(g["cols"]).cuda()

            def relf():
                if g is None:
                    return None
                xr = Xr.index_select(0, rows).index_select(1, cols).cpu().numpy()
                xi = Xi.index_select(0, rows).index_select(1, cols).cpu().numpy()
                return float(np.sqrt(np.sum((xr - g["xr"]) ** 2 + (xi - g["xi"]) ** 2)
                                     / np.sum(g["xr"] ** 2 + g["xi"] ** 2)))
            for pname, prec, f32c in (("f64", fi.FROB_PREC_F64, False), ("f64_f32corr", fi.FROB_PREC_F64, True),
                                      ("f32", fi.FROB_PREC_F32, False), ("bf16", fi.FROB_PREC_BF16, False)):
                key = f"mp{n}_{kind}_k1e{kexp}_{pname}"
                entry = {"reference": "oracle band samples" if g is not None else None}
                try:
                    fn(h, dA, dB, Xr, Xi, prec=prec)
                    entry["relF_unrefined"] = relf()
                    res = {}

                    def run():
                        res.update(fn(h, dA, dB, Xr, Xi, prec=prec, refine=8, f32_correction=f32c)[2])
                    run()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    run()
                    torch.cuda.synchronize()
                    entry.update({"ms_refined": (time.perf_counter() - t0) * 1e3, "refine_steps": res["refine_steps"],
                                  "resid0": res["resid0"], "resid": res["resid"], "norm2_est": res["norm2_est"],
                                  "relF_refined": relf()})
                except fi.FrobError as e:
                    entry["status"] = str(e)
                out[key] = entry
                log(f"[bench] {key}: {entry}")
            del dA, dB
            torch.cuda.empty_cache()
    return out


def bench_large_order(fi, inputs, h, torch, np, log, n):
    """Frobenius against complex-LU inversion at order n (8192), same recipe
    as the headline matrix (A, B iid N(0, 1), seed 0): plain FP64, then one and
    two Newton-Schulz steps (FP32 and FP64 correction) until the error on the
    oracle's sampled columns (tests/golden/n<n>_general_samples.npz, when
    present) is <= 1e-10; the complex-LU baseline in getri and printed form.
    Two timed runs after one warm-up each."""
    A, B = inputs.general(n, 0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Xr = torch.empty_like(dA)
    Xi = torch.empty_like(dA)
    gold = os.path.join(ROOT, "tests", "golden", f"n{n}_general_samples.npz")
    g = np.load(gold, allow_pickle=False) if os.path.exists(gold) else None

    def relf():
        if g is None:
            return None
        gc = g["cols"]
        gr, gi = Xr[:, gc].cpu().numpy(), Xi[:, gc].cpu().numpy()
        return float(np.sqrt(np.sum((gr - g["xr"]) ** 2 + (gi - g["xi"]) ** 2) / np.sum(g["xr"] ** 2 + g["xi"] ** 2)))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / 2 * 1e3

    out = {"n": n, "gold_samples": g is not None}
    log(f"[bench] n={n}: frobenius plain")
    out["frobenius_plain_ms"] = timed(lambda: fi.frob_inv_general(h, dA, dB, Xr, Xi))
    out["frobenius_plain_relF"] = relf()
    best = None
    if out["frobenius_plain_relF"] is not None and out["frobenius_plain_relF"] <= 1e-10:
        best = ("plain", out["frobenius_plain_ms"])
    for r in (1, 2):
        if best is not None:
            break
        for f32c in (True, False):
            tag = f"frobenius_refine{r}{'_f32corr' if f32c else ''}"
            log(f"[bench] n={n}: {tag}")
            ms = timed(lambda: fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=r, final_resid=False,
                                                   f32_correction=f32c))
            e = relf()
            out[tag + "_ms"], out[tag + "_relF"] = ms, e
            if e is not None and e <= 1e-10 and (best is None or ms < best[1]):
                best = (tag, ms)
    for form in (1, 0):
        log(f"[bench] n={n}: complex LU form {form}")
        out[f"complex_lu_form{form}_ms"] = timed(lambda: fi.frob_cinv_lu(h, dA, dB, Xr, Xi, form=form))
        out[f"complex_lu_form{form}_relF"] = relf()
    if best is not None:
        out["frobenius_at_1e-10"] = {"config": best[0], "ms": best[1]}
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()
    return {f"n{n}_frobenius_vs_complex_lu": out}


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

    if args.batched_only:
        h = fi.Handle(0)
        print(json.dumps(bench_batched(fi, inputs, h, torch, np, log, tune=False, loop=False)), flush=True)
        return
    if args.adjoint_only:
        h = fi.Handle(0)
        print(json.dumps(bench_adjoint(fi, inputs, h, torch, np, log)), flush=True)
        return

    n, K, W = args.n, args.steps, args.warmup
    torch.cuda.set_device(0)
    log(f"[bench] generating inputs n={n}")
    A, B = inputs.general(n, 0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Xr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    Xi = torch.empty_like(Xr)
    h = fi.Handle(0)

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    def measure(fn):
        """W warm-up steps, then K timed steps with the library's kernel
        profiling on: HIP events on the library's stream around the n x n x n
        GEMMs, and on its second stream around the look-ahead LUs'
        trailing-update GEMMs."""
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        h.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            fn()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / K
        prof = {"nnn": h.profile_read(0), "trail": h.profile_read(6)}
        h.profile(False)
        return t, prof

    def relf_gold(kind):
        """relative Frobenius error of the current X on the oracle's sampled columns"""
        gold = os.path.join(ROOT, "tests", "golden", f"n{n}_{kind}_samples.npz")
        if not os.path.exists(gold):
            return None
        g = np.load(gold, allow_pickle=False)
        gc = g["cols"]
        gr, gi = Xr[:, gc].cpu().numpy(), Xi[:, gc].cpu().numpy()
        return float(np.sqrt(np.sum((gr - g["xr"]) ** 2 + (gi - g["xi"]) ** 2) /
                             np.sum(g["xr"] ** 2 + g["xi"] ** 2)))

    def backward_error():
        """||M x_j - e_j|| / (||M|| ||x_j||) on seeded sampled columns"""
        rng = np.random.default_rng(123)
        cols = np.sort(rng.choice(n, size=min(8, n), replace=False))
        xr = Xr[:, cols].cpu().numpy()
        xi = Xi[:, cols].cpu().numpy()
        E = np.zeros((n, len(cols)))
        E[cols, np.arange(len(cols))] = 1.0
        Rr = A @ xr - B @ xi - E
        Ri = A @ xi + B @ xr
        normM = np.linalg.norm(A, 2) if n <= 2048 else np.sqrt(np.sum(A * A) + np.sum(B * B))
        return float(np.sqrt(np.sum(Rr ** 2 + Ri ** 2)) / (normM * np.sqrt(np.sum(xr ** 2 + xi ** 2))))

    # Plain FP64 Frobenius inversion, then (when its error against the oracle
    # exceeds the metric's 1e-10) the cheapest refined configuration that
    # reaches it: the timed headline is time-to-solution at rel err <= 1e-10.
    log(f"[bench] frobenius general (plain FP64): warmup {W}, steps {K}")
    t_plain, prof_plain = measure(lambda: fi.frob_inv_general(h, dA, dB, Xr, Xi))
    err_plain = relf_gold("general")
    berr_plain = backward_error()
    log(f"[bench] plain: {t_plain * 1e3:.3f} ms/step, relF vs oracle {err_plain}")
    chosen = {"refine": 0, "t": t_plain, "prof": prof_plain, "err": err_plain, "berr": berr_plain}
    # Refined candidates: r steps with the correction X R in FP64 or in FP32
    # (residual FP64 in both); the fastest that reaches 1e-10 at the smallest r.
    trials = []
    if err_plain is not None and err_plain > 1e-10:
        for r in (1, 2):
            for f32c in (True, False):
                tag = f"refine={r}{' f32-correction' if f32c else ''}"
                log(f"[bench] frobenius general, {tag}: warmup {W}, steps {K}")
                t_r, prof_r = measure(lambda: fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=r, final_resid=False,
                                                                  f32_correction=f32c))
                err_r = relf_gold("general")
                log(f"[bench] {tag}: {t_r * 1e3:.3f} ms/step, relF vs oracle {err_r}")
                trials.append({"refine": r, "f32_correction": f32c, "ms": t_r * 1e3, "relF_vs_oracle_sampled_cols": err_r})
                if err_r is not None and err_r <= 1e-10 and (chosen["refine"] == 0 or t_r < chosen["t"]):
                    chosen = {"refine": r, "f32c": f32c, "t": t_r, "prof": prof_r, "err": err_r,
                              "berr": backward_error()}
            if chosen["refine"]:
                break
    t_step = chosen["t"]
    berr, relf_samples = chosen["berr"], chosen["err"]

    extra = {"plain_fp64": {"ms": t_plain * 1e3, "relF_vs_oracle_sampled_cols": err_plain,
                            "backward_error_sampled_cols": berr_plain},
             "refine_trials": trials}
    if not args.no_extra:
        log("[bench] frobenius HPD")
        Ah, Bh = inputs.hpd(n, 1)
        dAh, dBh = torch.from_numpy(Ah).cuda(), torch.from_numpy(Bh).cuda()
        t_hpd = timed(lambda: fi.frob_inv_hpd(h, dAh, dBh, Xr, Xi), max(2, K // 2), 1)
        extra["hpd_ms"] = t_hpd * 1e3
        extra["hpd_inversions_per_s"] = 1.0 / t_hpd
        extra["hpd_eff_tflops_4n3"] = 4.0 * n ** 3 / t_hpd / 1e12
        extra["hpd_relF_vs_oracle_sampled_cols"] = relf_gold("hpd")
        for name, fn, Mr, Mi, kind in (("cinv_lu", fi.frob_cinv_lu, dA, dB, "general"),
                                       ("cinv_chol", fi.frob_cinv_chol, dAh, dBh, "hpd")):
            for form in (1, 0):
                try:
                    t = timed(lambda: fn(h, Mr, Mi, Xr, Xi, form=form), max(2, K // 2), 1)
                    extra[f"{name}_form{form}_ms"] = t * 1e3
                    extra[f"{name}_form{form}_relF_vs_oracle_sampled_cols"] = relf_gold(kind)
                except fi.FrobError as e:
                    extra[f"{name}_form{form}_ms"] = None
                    log(f"[bench] {name} form {form} unavailable: {e}")
        # mixed precision + Newton-Schulz (same general and HPD matrices)
        for tag, fn, Ma, Mb, kind in (("mp_general", fi.frob_inv_general, dA, dB, "general"),
                                      ("mp_hpd", fi.frob_inv_hpd, dAh, dBh, "hpd")):
            for pname, prec in (("f32", fi.FROB_PREC_F32), ("bf16", fi.FROB_PREC_BF16)):
                key = f"{tag}_{pname}"
                log(f"[bench] {key}")
                try:
                    res = {}

                    def run_mp():
                        res.update(fn(h, Ma, Mb, Xr, Xi, prec=prec, refine=8)[2])
                    t = timed(run_mp, 2, 1)
                    extra[key] = {"ms": t * 1e3, "refine_steps": res["refine_steps"], "resid0": res["resid0"],
                                  "resid": res["resid"], "relF_vs_oracle_sampled_cols": relf_gold(kind)}
                except fi.FrobError as e:
                    extra[key] = {"status": str(e)}
        del dAh, dBh
        extra.update(bench_batched(fi, inputs, h, torch, np, log))
        extra.update(bench_adjoint(fi, inputs, h, torch, np, log))
        if not args.no_newton:
            extra.update(bench_newton(fi, inputs, h, torch, np, log))
        if not args.no_mp_large or not args.no_large:
            del Xr, Xi
            torch.cuda.empty_cache()
        if not args.no_large:
            extra.update(bench_large_order(fi, inputs, h, torch, np, log, 8192))
        if not args.no_mp_large:
            extra.update(bench_mp_large(fi, inputs, h, torch, np, log, args.mp_n))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # bounded sample: Algorithm 5 of the FP64 oracle on all host threads at
        # n = cpu_n, and on one thread at n = cpu_n / 2, each scaled by n^3
        m = min(args.cpu_n, n)
        Ac, Bc = inputs.general(m, 0)
        threads = oracle.num_threads()
        log(f"[bench] cpu baseline: oracle Algorithm 5 at n={m}, {threads} threads")
        tc0 = time.perf_counter()
        oracle.frob_lu(Ac, Bc)
        tc = time.perf_counter() - tc0
        m1 = max(1, (3 * m) // 8)
        A1, B1 = inputs.general(m1, 0)
        log(f"[bench] cpu baseline: oracle Algorithm 5 at n={m1}, 1 thread")
        prev = oracle.set_num_threads(1)
        tc1_0 = time.perf_counter()
        oracle.frob_lu(A1, B1)
        tc1 = time.perf_counter() - tc1_0
        oracle.set_num_threads(prev)
        cpu = {"value": 1.0 / (tc * (n / m) ** 3), "unit": "inversions/s", "cores": threads, "kind": "oracle",
               "sample": f"one n={m} general matrix of the same recipe (seed 0), Algorithm 5 in the FP64 oracle on "
                         f"{threads} threads, {tc:.2f} s, scaled to n={n} by (n/{m})^3",
               "single_thread_value": 1.0 / (tc1 * (n / m1) ** 3),
               "single_thread_sample": f"n={m1}, 1 thread, {tc1:.2f} s, scaled by (n/{m1})^3"}
        if args.cpu_full and m < n:
            log(f"[bench] cpu baseline: oracle Algorithm 5 at the full order n={n}, {threads} threads")
            tf0 = time.perf_counter()
            oracle.frob_lu(A, B)
            tf = time.perf_counter() - tf0
            cpu["full_size_value"] = 1.0 / tf
            cpu["full_size_sample"] = f"one run at n={n} on {threads} threads, {tf:.1f} s"

    comparison = None
    if "cinv_lu_form1_ms" in extra:
        comparison = {"frobenius_ms_at_1e-10": t_step * 1e3, "frobenius_refine_steps": chosen["refine"],
                      "frobenius_f32_correction": chosen.get("f32c", False),
                      "complex_lu_getri_form_ms": extra["cinv_lu_form1_ms"],
                      "complex_lu_getri_form_relF": extra.get("cinv_lu_form1_relF_vs_oracle_sampled_cols"),
                      "complex_lu_printed_form_ms": extra.get("cinv_lu_form0_ms"),
                      "complex_lu_printed_form_relF": extra.get("cinv_lu_form0_relF_vs_oracle_sampled_cols")}

    def roof(cls, kernel, traffic_file, sources):
        launches, ms, flops, nbytes = chosen["prof"][cls]
        if not launches:
            return None
        avg_ms = ms / launches
        achieved = flops / (ms * 1e-3) / 1e12
        intensity = flops / nbytes if nbytes else None
        ridge = FP64_MFMA_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        # HBM traffic from the committed rocprofv3 counter summary, valid only
        # while the kernel's sources are the ones measured
        traffic = None
        tj = os.path.join(ROOT, "profiles", traffic_file)
        if n == 4096 and os.path.exists(tj):
            import hashlib
            with open(tj) as f:
                td = json.load(f)
            ok = True
            for src, key in sources:
                with open(os.path.join(ROOT, "paper_2208_01239_amd", "csrc", src), "rb") as f:
                    ok = ok and hashlib.sha256(f.read()).hexdigest() == td.get(key)
            if ok:
                traffic = td["traffic_bytes_per_launch"]
        common = {"kernel": kernel, "traffic": traffic, "avg_launch_ms": avg_ms, "launches_per_step": launches / K,
                  "alg_flops_per_launch": flops / launches, "alg_bytes_per_launch": nbytes / launches,
                  "intensity_flop_per_byte": intensity, "fp64_ridge_flop_per_byte": ridge,
                  "mfma_tflops": achieved, "mfma_frac": achieved / FP64_MFMA_PEAK_TFLOPS,
                  "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)"}
        if intensity is not None and intensity < ridge:
            gbs = nbytes / (ms * 1e-3) / 1e9     # below the ridge: the HBM roof bounds the kernel
            return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                    **common}
        return {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_MFMA_PEAK_TFLOPS, **common}

    roof_trail = roof("trail", "k_gemm_f64 persistent (capped grid): trailing-update GEMMs of the look-ahead LUs of A "
                      "and C on the second stream, 2 m w k flops per launch",
                      "gemm_f64_trailing_n4096_hbm_traffic.json",
                      [("gemm_f64.hip", "gemm_f64_hip_sha256"), ("lu_f64.hip", "lu_f64_hip_sha256")])
    roof_nnn = roof("nnn", "k_gemm_f64<128,128>: the n x n x n products B*Y and -Y*C^-1, 2 n^3 flops per launch",
                    "gemm_f64_128x128_n4096_hbm_traffic.json", [("gemm_f64.hip", "gemm_f64_hip_sha256")])
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
        "dtype": "f64 (Newton-Schulz correction f32)" if chosen.get("f32c") else "f64",
        "data": "synthetic",
        "config": {"workload": f"frobenius_general_n{n}_fp64", "n": n, "generator": "A,B iid N(0,1) seed 0",
                   "batch": 1, "newton_schulz_steps": chosen["refine"],
                   "newton_schulz_f32_correction": chosen.get("f32c", False),
                   "accuracy": "rel. Frobenius error vs the FP64 oracle on sampled columns <= 1e-10"},
        "eff_tflops_8n3": 8.0 * n ** 3 / t_step / 1e12,
        "relF_vs_oracle_sampled_cols": relf_samples,
        "roofline": roof_trail if roof_trail is not None else roof_nnn,
        "roofline_nnn": roof_nnn,
        "cpu_baseline": cpu,
    }
    if "cinv_lu_form1_ms" in extra:
        line["complex_lu_ms"] = {"getri": extra["cinv_lu_form1_ms"], "printed": extra.get("cinv_lu_form0_ms")}
        line["frobenius_plain_ms"] = t_plain * 1e3
        line["frobenius_plain_relF"] = err_plain
        line["hpd_ms"] = {"frobenius": extra.get("hpd_ms"), "complex_chol_potri": extra.get("cinv_chol_form1_ms"),
                          "complex_chol_printed": extra.get("cinv_chol_form0_ms")}
    detail = dict(line)
    detail["backward_error_sampled_cols"] = berr
    detail["alg_tflops_26n3_3"] = (26.0 / 3.0) * n ** 3 / t_step / 1e12
    detail["frobenius_vs_complex_lu"] = comparison
    detail.update(extra)
    out_dir = os.path.join(ROOT, "gpurun_out")
    try:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "bench_detail.json"), "w") as f:
            json.dump(detail, f, indent=1)
        log(f"[bench] details written to {os.path.join(out_dir, 'bench_detail.json')}")
    except OSError as e:
        log(f"[bench] details not written: {e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
