"""Oracle values at a few sites of a lattice too large for the oracle.

TEST INFRASTRUCTURE: only the tests use this module.

Every operator of the library is a product of nearest-neighbour hops and
site-local fifth-dimension matrices.  Its output at site c therefore depends
only on the input within taxicab distance r of c (r = number of hops) and on
the links whose base site lies in that ball.  These values are copied into a
small periodic frame lattice of extent 2r + 2 in every direction, with c at
the frame centre and the parity of every site kept, and zeros elsewhere; the
FP64 oracle applied to the frame gives, at the frame centre, the operator's
output at c.  In the frame no hop that matters crosses a boundary, so the time
boundary condition of the big lattice is folded into the copied input: a site
reached from c by crossing the time boundary k times carries the factor bc_t**k
(a site-dependent sign change that commutes with every site-local matrix and
turns each boundary-crossing hop of the big lattice into a plain hop).
"""
import numpy as np

from oracle import oracle

RADIUS = {
    oracle.OP_HOP_EO: 1, oracle.OP_HOP_OE: 1, oracle.OP_M5INV: 0, oracle.OP_D: 1,
    oracle.OP_DDAG: 1, oracle.OP_DDAGD: 2, oracle.OP_SCHUR: 2, oracle.OP_SCHUR_DAG: 2,
    oracle.OP_SCHUR_NORMAL: 4,
}
# parity of the sites where an operator's output lives (None: every site)
OUT_PARITY = {
    oracle.OP_HOP_EO: 0, oracle.OP_HOP_OE: 1, oracle.OP_SCHUR: 0, oracle.OP_SCHUR_DAG: 0,
    oracle.OP_SCHUR_NORMAL: 0,
}


def ball(r):
    """All offsets (dx, dy, dz, dt) with |dx| + |dy| + |dz| + |dt| <= r."""
    rng = np.arange(-r, r + 1)
    d = np.stack(np.meshgrid(rng, rng, rng, rng, indexing="ij"), -1).reshape(-1, 4)
    return d[np.abs(d).sum(1) <= r]


def pick_sites(dims, n, parity, seed):
    """n sites (x, y, z, t) of the given parity (None: any): the lattice corners
    and faces first (both time boundaries, x = 0 and x = X - 1, ...), then
    random sites from default_rng(seed)."""
    X, Y, Z, T = dims
    cand = [(0, 0, 0, 0), (X - 1, Y - 1, Z - 1, T - 1), (1, 2, 3, 0), (X - 1, 0, Z - 1, T - 1),
            (0, Y - 1, 0, T - 1), (X - 2, 1, 0, 0), (X // 2, Y // 2, Z // 2, T // 2)]
    rng = np.random.default_rng(seed)
    while len(cand) < 4 * n + 16:
        cand.append(tuple(int(rng.integers(L)) for L in dims))
    out = []
    for c in cand:
        if parity is not None and sum(c) % 2 != parity:
            c = ((c[0] + 1) % X,) + tuple(c[1:])
            if X % 2 and sum(c) % 2 != parity:  # odd extents have no clean parity
                continue
        if c not in out:
            out.append(c)
        if len(out) == n:
            break
    return out


def frame(site, dims, r, bc_t):
    """Copy plan for one site: (source coordinates [n, 4], factors [n],
    frame coordinates [n, 4], frame extent F)."""
    F = max(2 * r + 2, 2)
    c0 = np.array([r + 1] * 4)
    c = np.asarray(site)
    if (c0.sum() - c.sum()) % 2:
        c0[0] = (c0[0] + 1) % F  # keep the parity of every copied site
    d = ball(r)
    u = c[None, :] + d                      # unwrapped coordinates
    L = np.asarray(dims)
    src = u % L
    wraps = np.floor_divide(u[:, 3], L[3])  # signed number of time-boundary crossings
    fac = np.where(wraps % 2 == 0, 1.0, float(bc_t))
    dst = (c0[None, :] + d) % F
    return src, fac, dst, F, c0


def oracle_at_sites(op, sites, dims, bc_t, get_psi, get_U, Ns, m0, omega, mu):
    """FP64 oracle output of `op` at each site (x, y, z, t) of `sites`.

    get_psi(coords[n, 4]) -> complex128 [Ns][n][4][3]   input at those sites
    get_U(coords[n, 4])   -> complex128 [n][4][3][3]    U_mu at those sites
    returns complex128 [len(sites)][Ns][4][3]
    """
    r = RADIUS[op]
    out = []
    for site in sites:
        src, fac, dst, F, c0 = frame(site, dims, r, bc_t)
        psi_f = np.zeros((Ns, F, F, F, F, 4, 3), np.complex128)
        U_f = np.zeros((F, F, F, F, 4, 3, 3), np.complex128)
        p = np.asarray(get_psi(src)) * fac[None, :, None, None]
        U = np.asarray(get_U(src))
        x, y, z, t = dst[:, 0], dst[:, 1], dst[:, 2], dst[:, 3]
        psi_f[:, t, z, y, x] = p
        U_f[t, z, y, x] = U
        o = oracle.apply(op, U_f, psi_f, m0, omega, mu, bc_t=1)
        out.append(o[:, c0[3], c0[2], c0[1], c0[0]])
    return np.stack(out)


def numpy_getters(psi, U):
    """Getters over full host arrays psi[s][t][z][y][x][4][3], U[t][z][y][x][mu][3][3]."""
    def gp(c):
        return psi[:, c[:, 3], c[:, 2], c[:, 1], c[:, 0]]

    def gu(c):
        return U[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]
    return gp, gu


def torch_getters(psi, U):
    """Getters over device tensors (same layouts); only the gathered values
    are copied to the host."""
    import torch

    def idx(c):
        return [torch.as_tensor(c[:, k], device=psi.device, dtype=torch.long) for k in (3, 2, 1, 0)]

    def gp(c):
        t, z, y, x = idx(c)
        return psi[:, t, z, y, x].cpu().numpy()

    def gu(c):
        t, z, y, x = idx(c)
        return U[t, z, y, x].cpu().numpy()
    return gp, gu


def at_sites(field, sites):
    """field[s][t][z][y][x][4][3] (numpy or torch) at the sites -> numpy [n][Ns][4][3]."""
    c = np.asarray(sites)
    if isinstance(field, np.ndarray):
        v = field[:, c[:, 3], c[:, 2], c[:, 1], c[:, 0]]
    else:
        import torch
        ix = [torch.as_tensor(c[:, k], device=field.device, dtype=torch.long) for k in (3, 2, 1, 0)]
        v = field[:, ix[0], ix[1], ix[2], ix[3]].cpu().numpy()
    return np.moveaxis(v, 1, 0)
