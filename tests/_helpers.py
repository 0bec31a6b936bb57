"""Shared helpers for the test suite (metrics and device transfer)."""
import numpy as np


def relF(Xr, Xi, Rr, Ri):
    """Relative Frobenius error over both parts: ||X - R||_F / ||R||_F."""
    Xr, Xi, Rr, Ri = (np.asarray(a, dtype=np.float64) for a in (Xr, Xi, Rr, Ri))
    return float(np.sqrt(np.sum((Xr - Rr) ** 2 + (Xi - Ri) ** 2) / np.sum(Rr ** 2 + Ri ** 2)))


def maxnorm(Xr, Xi):
    """Complex max norm of eq. (maxnorm): max over both parts."""
    return float(max(np.abs(Xr).max(), np.abs(Xi).max()))


def res_left(Mr, Mi, Yr, Yi):
    """res_L of eq. (backerr): ||Y X - I||_max / (||X||_max ||Y||_max)."""
    M = Mr + 1j * Mi
    Y = Yr + 1j * Yi
    R = Y @ M - np.eye(M.shape[0])
    return maxnorm(R.real, R.imag) / (maxnorm(Mr, Mi) * maxnorm(Yr, Yi))


def res_right(Mr, Mi, Yr, Yi):
    M = Mr + 1j * Mi
    Y = Yr + 1j * Yi
    R = M @ Y - np.eye(M.shape[0])
    return maxnorm(R.real, R.imag) / (maxnorm(Mr, Mi) * maxnorm(Yr, Yi))


def to_dev(a, ld=None):
    """float64 numpy -> torch cuda tensor, optionally with a padded leading dimension."""
    import torch
    a = np.array(a, dtype=np.float64, order="C", copy=True)   # fresh, standard strides (also for 1 x 1 views)
    if ld is None or ld == a.shape[1]:
        return torch.from_numpy(a).cuda()
    buf = torch.full((a.shape[0], ld), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, : a.shape[1]] = torch.from_numpy(a).cuda()
    return buf[:, : a.shape[1]]


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)
