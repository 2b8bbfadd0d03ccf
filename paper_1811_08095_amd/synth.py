"""Seeded synthetic inputs: SU(3) gauge fields and Gaussian sources.

This module holds no part of the operator or the solver; it only draws the
inputs that both the library and the oracle consume, so that the two see
identical bits.  The paper's thermalised beta = 6.20 ensembles (§2) are not
available; these fields stand in for them.

Gauge links: U_mu(x) = exp(i eps H), H = sum_a h_a lambda_a / 2 with the
Gell-Mann matrices lambda_a and h_a ~ N(0, 1) iid, drawn from
numpy.random.default_rng(seed).standard_normal((T, Z, Y, X, 4, 8)) in C order
(the draw is streamed in t-slices; the sequence is the same as one call).
Sources: Re, Im ~ N(0, 1) iid from default_rng(seed), canonical order
[rhs][s][t][z][y][x][spin][color][re/im].
"""
import numpy as np

try:  # torch's batched matrix exponential is the fastest exp available here
    import torch
except ImportError:  # pragma: no cover
    torch = None


def gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    return lam


def _expi(Hs: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices."""
    A = 1j * eps * Hs
    if torch is not None:
        return torch.linalg.matrix_exp(torch.from_numpy(A)).numpy()
    w, V = np.linalg.eigh(Hs)
    return (V * np.exp(1j * eps * w)[..., None, :]) @ np.swapaxes(V.conj(), -1, -2)


def make_gauge(dims, eps: float, seed: int, out: np.ndarray = None) -> np.ndarray:
    """Gauge field U[t][z][y][x][mu][3][3] (complex128) for dims = (X, Y, Z, T)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    lam = gell_mann() * 0.5
    if out is None:
        out = np.empty((T, Z, Y, X, 4, 3, 3), np.complex128)
    for t in range(T):
        h = rng.standard_normal((Z, Y, X, 4, 8))
        H = np.tensordot(h, lam, axes=([4], [0]))          # [Z,Y,X,4,3,3]
        H = 0.5 * (H + np.swapaxes(H.conj(), -1, -2))      # exact hermiticity
        out[t] = _expi(H.reshape(-1, 3, 3), eps).reshape(Z, Y, X, 4, 3, 3)
    return out


def make_source(dims, Ns: int, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian sources b[rhs][s][t][z][y][x][4][3] (complex128)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((nrhs, Ns, T, Z, Y, X, 4, 3, 2))
    return r[..., 0] + 1j * r[..., 1]


def unit_gauge(dims) -> np.ndarray:
    X, Y, Z, T = (int(d) for d in dims)
    U = np.zeros((T, Z, Y, X, 4, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


# ---------------------------------------------------------------------------
# device-side generators for lattices too large to draw on the host in
# reasonable time (64^4 x 16 sources hold 3.2e9 complex numbers).  Same
# distributions; the stream is torch's seeded device generator (Philox), drawn
# in t-slices in the canonical order.
# ---------------------------------------------------------------------------

def make_gauge_device(dims, eps: float, seed: int, device="cuda"):
    """U = exp(i eps H) as a complex128 CUDA tensor [t][z][y][x][4][3][3]."""
    import torch
    X, Y, Z, T = (int(d) for d in dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    lam = torch.from_numpy((gell_mann() * 0.5).reshape(8, 9)).to(device)
    out = torch.empty((T, Z, Y, X, 4, 3, 3), dtype=torch.complex128, device=device)
    for t in range(T):
        h = torch.randn((Z * Y * X * 4, 8), generator=g, device=device, dtype=torch.float64)
        H = (h.to(torch.complex128) @ lam).reshape(-1, 3, 3)
        H = 0.5 * (H + H.transpose(-1, -2).conj())
        out[t] = torch.linalg.matrix_exp(1j * eps * H).reshape(Z, Y, X, 4, 3, 3)
    return out


def make_source_device(dims, Ns: int, nrhs: int, seed: int, device="cuda"):
    """Complex Gaussian source (Re, Im ~ N(0,1)) as a CUDA tensor
    [rhs][s][t][z][y][x][4][3]."""
    import torch
    X, Y, Z, T = (int(d) for d in dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((nrhs, Ns, T, Z, Y, X, 4, 3), dtype=torch.complex128, device=device)
    v = torch.view_as_real(out)
    for r in range(nrhs):
        for s in range(Ns):
            v[r, s].normal_(generator=g)
    return out
