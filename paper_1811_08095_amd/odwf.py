"""Thin ctypes binding of libodwf.so (include/odwf.h).

Argument marshalling only: every step of the operator and the solvers runs in
the library's HIP kernels.  PyTorch provides device memory (complex128 CUDA
tensors) and streams; numpy arrays are accepted where the ABI takes host
memory (gauge upload, weights).  The binding raises if the library has not
been built: there is no fallback path.

Canonical layouts (identical to the C ABI):
  gauge   U[t][z][y][x][mu][3][3]          complex128
  spinor  psi[rhs][s][t][z][y][x][4][3]     complex128 (device)
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ODWF_LIB selects another build of the library (tuning builds); default in-tree
LIBPATH = os.environ.get("ODWF_LIB") or os.path.join(HERE, "libodwf.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENAN, EBUSY = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, FP16S, BF16S = 0, 1, 2, 3
OP_HOP_EO, OP_HOP_OE, OP_M5INV, OP_D, OP_DDAG, OP_DDAGD, OP_SCHUR, OP_SCHUR_DAG, \
    OP_SCHUR_NORMAL = range(9)
SOLVE_EO_NORMAL, SOLVE_FULL = 0, 1
PREC_NAMES = {FP64: "fp64", FP32: "fp32", FP16S: "fp16s", BF16S: "bf16s"}


class OdwfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"odwf status {status}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("outer_steps", ctypes.c_int), ("status", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("full_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

SYMBOLS = {
    "odwf_lattice_create": ([ctypes.POINTER(ctypes.c_int), _i, _i, ctypes.POINTER(_vp)], _i),
    "odwf_lattice_load_gauge": ([_vp, _vp, _i, _vp], _i),
    "odwf_lattice_bytes": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _i),
    "odwf_lattice_destroy": ([_vp], None),
    "odwf_solver_create": ([_vp, _i, _d, _dp, ctypes.POINTER(_vp)], _i),
    "odwf_solver_destroy": ([_vp], None),
    "odwf_apply": ([_vp, _i, _dp, _i, _i, _vp, _vp, _vp], _i),
    "odwf_apply_noalloc": ([_vp, _i, _dp, _i, _i, _vp, _vp, _vp], _i),
    "odwf_solve": ([_vp, _i, _dp, _dp, _i, _i, _i, _vp, _vp, _i, ctypes.POINTER(Stats), _vp], _i),
    "odwf_solver_reserve": ([_vp, _i, _i, _vp], _i),
    "odwf_force": ([_vp, _vp, _vp, _i, _vp, _vp], _i),
    "odwf_deff": ([_vp, _i, _dp, _dp, _i, _i, _i, _vp, _vp, ctypes.POINTER(Stats), _vp], _i),
    "odwf_solve_masses": ([_vp, _dp, _dp, _i, _i, _i, _vp, _vp, _i, _i, ctypes.POINTER(Stats), _vp], _i),
    "odwf_footprint": ([ctypes.POINTER(ctypes.c_int), _i, _i, _i, ctypes.POINTER(ctypes.c_size_t)], _i),
    "odwf_zolotarev_omega": ([_i, _d, _d, _dp], _i),
    "odwf_batch_create": ([_vp, _i, _i, ctypes.POINTER(_vp)], _i),
    "odwf_batch_admit": ([_vp, _vp, _d, _d, _i, _ip, _vp], _i),
    "odwf_batch_step": ([_vp, _i, _vp], _i),
    "odwf_batch_poll": ([_vp, _i, _ip, ctypes.POINTER(Stats), _vp], _i),
    "odwf_batch_retire": ([_vp, _i, _vp, ctypes.POINTER(Stats), _vp], _i),
    "odwf_batch_free_slots": ([_vp, _ip], _i),
    "odwf_batch_footprint": ([ctypes.POINTER(ctypes.c_int), _i, _i, _i, ctypes.POINTER(ctypes.c_size_t)], _i),
    "odwf_batch_bytes": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _i),
    "odwf_batch_destroy": ([_vp], None),
    "odwf_profile_enable": ([_i], _i),
    "odwf_profile_read": ([ctypes.POINTER(ctypes.c_longlong), _dp, _dp], _i),
    "odwf_profile_read_kernel": ([_i, _i, ctypes.POINTER(ctypes.c_longlong), _dp, _dp], _i),
    "odwf_last_error": ([], ctypes.c_char_p),
    "odwf_version": ([], ctypes.c_char_p),
}


def lib():
    """Open libodwf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBPATH)
        for name, (args, res) in SYMBOLS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st, allow=()):
    if st != OK and st not in allow:
        raise OdwfError(st, lib().odwf_last_error().decode())
    return st


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _dims_arr(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def _f64arr(vals):
    a = np.ascontiguousarray(np.asarray(vals, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(_dp)


def _dev_ptr(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous complex128 tensor")
    return _vp(t.data_ptr())


def version():
    return lib().odwf_version().decode()


def zolotarev_omega(Ns, lmin=0.05, lmax=6.2):
    """Optimal weights omega_s (host computation in the library)."""
    out = np.zeros(Ns, np.float64)
    _check(lib().odwf_zolotarev_omega(int(Ns), float(lmin), float(lmax), out.ctypes.data_as(_dp)))
    return out


def footprint(dims, Ns, nrhs, inner):
    b = ctypes.c_size_t()
    _check(lib().odwf_footprint(_dims_arr(dims), int(Ns), int(nrhs), int(inner), ctypes.byref(b)))
    return b.value


def batch_footprint(dims, Ns, max_slots, inner):
    """Device bytes of a batch engine of max_slots slots (odwf_batch_footprint)."""
    b = ctypes.c_size_t()
    _check(lib().odwf_batch_footprint(_dims_arr(dims), int(Ns), int(max_slots), int(inner), ctypes.byref(b)))
    return b.value


def profile_enable(on=True):
    _check(lib().odwf_profile_enable(1 if on else 0))


def profile_read():
    """(launches, milliseconds, algorithmic bytes) of the hopping kernels."""
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(lib().odwf_profile_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def profile_read_kernel(prec, dag):
    """(launches, milliseconds, algorithmic bytes) of one hopping-kernel
    instantiation: storage precision prec, dag 0 (W) or 1 (W^dag)."""
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(lib().odwf_profile_read_kernel(int(prec), int(dag), ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(by)))
    return n.value, ms.value, by.value


class Lattice:
    def __init__(self, dims, bc_t=-1, device=0):
        self.dims = tuple(int(d) for d in dims)  # (X, Y, Z, T)
        self.bc_t = int(bc_t)
        h = _vp()
        _check(lib().odwf_lattice_create(_dims_arr(self.dims), self.bc_t, int(device), ctypes.byref(h)))
        self._h = h

    @property
    def shape_tzyx(self):
        X, Y, Z, T = self.dims
        return (T, Z, Y, X)

    def load_gauge(self, U, stream=None):
        """U: numpy (host) or torch CUDA complex128 [t][z][y][x][4][3][3]."""
        try:
            import torch
            is_t = isinstance(U, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_t = False
        if is_t:
            ptr, on_dev = _dev_ptr(U, "U"), 1
            keep = U
        else:
            keep = np.ascontiguousarray(U, dtype=np.complex128)
            if keep.shape != self.shape_tzyx + (4, 3, 3):
                raise ValueError("gauge field has the wrong shape")
            ptr, on_dev = _vp(keep.ctypes.data), 0
        _check(lib().odwf_lattice_load_gauge(self._h, ptr, on_dev, _stream(stream)))
        del keep

    def nbytes(self):
        b = ctypes.c_size_t()
        _check(lib().odwf_lattice_bytes(self._h, ctypes.byref(b)))
        return b.value

    def close(self):
        if self._h:
            lib().odwf_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    def __init__(self, lattice, Ns, m0, omega):
        self.lattice = lattice
        self.Ns = int(Ns)
        self.m0 = float(m0)
        self.omega = np.ascontiguousarray(omega, np.float64)
        h = _vp()
        _check(lib().odwf_solver_create(lattice._h, self.Ns, self.m0,
                                        self.omega.ctypes.data_as(_dp), ctypes.byref(h)))
        self._h = h

    def spinor_shape(self, nrhs):
        return (nrhs, self.Ns) + self.lattice.shape_tzyx + (4, 3)

    def apply(self, op, psi, mq, prec=FP64, out=None, stream=None):
        import torch
        nrhs = psi.shape[0]
        if tuple(psi.shape) != self.spinor_shape(nrhs):
            raise ValueError("spinor has the wrong shape")
        if out is None:
            out = torch.empty_like(psi)
        mqa, mqp = _f64arr(np.broadcast_to(np.asarray(mq, np.float64), (nrhs,)))
        _check(lib().odwf_apply(self._h, int(op), mqp, int(prec), nrhs, _dev_ptr(psi, "in"),
                                _dev_ptr(out, "out"), _stream(stream)))
        return out

    def apply_noalloc(self, op, psi, mq, prec=FP64, out=None, stream=None):
        """odwf_apply_noalloc: the same operator with no device allocation in the
        call (`out`, when not given, is allocated here by torch beforehand)."""
        import torch
        nrhs = psi.shape[0]
        if tuple(psi.shape) != self.spinor_shape(nrhs):
            raise ValueError("spinor has the wrong shape")
        if out is None:
            out = torch.empty_like(psi)
        mqa, mqp = _f64arr(np.broadcast_to(np.asarray(mq, np.float64), (nrhs,)))
        _check(lib().odwf_apply_noalloc(self._h, int(op), mqp, int(prec), nrhs, _dev_ptr(psi, "in"),
                                        _dev_ptr(out, "out"), _stream(stream)))
        return out

    def solve(self, b, mq, tol=1e-10, mode=SOLVE_FULL, inner=FP64, maxiter=100000, x=None,
              use_x0=False, stream=None, raise_on_noconv=True):
        import torch
        nrhs = b.shape[0]
        if tuple(b.shape) != self.spinor_shape(nrhs):
            raise ValueError("source has the wrong shape")
        if x is None:
            x = torch.zeros_like(b)
        mqa, mqp = _f64arr(np.broadcast_to(np.asarray(mq, np.float64), (nrhs,)))
        tla, tlp = _f64arr(np.broadcast_to(np.asarray(tol, np.float64), (nrhs,)))
        stats = (Stats * nrhs)()
        st = lib().odwf_solve(self._h, int(mode), mqp, tlp, nrhs, int(inner), int(maxiter),
                              _dev_ptr(b, "b"), _dev_ptr(x, "x"), 1 if use_x0 else 0, stats,
                              _stream(stream))
        _check(st, allow=() if raise_on_noconv else (ENOCONV, ENAN))
        return x, [s.as_dict() for s in stats]

    def packed_even_shape(self, nrhs):
        """Shape of a packed even-half FP64 field of nrhs right-hand sides:
        [V/2 even sites][nrhs][12 spin-colour][Ns] complex128."""
        X, Y, Z, T = self.lattice.dims
        return (X * Y * Z * T // 2, nrhs, 12, self.Ns)

    def solve_masses(self, b, mq, tol=1e-10, inner=FP64, maxiter=100000, y=None, use_y0=False,
                     per_launch=0, stream=None, raise_on_noconv=True):
        """odwf_solve_masses: S_e(m_k)^dag S_e(m_k) y_k = b_e for every mass
        m_k of `mq`, one source b [Ns][t][z][y][x][4][3] (or [1][...]);
        per_launch masses per multi-right-hand-side CG (0: the library's choice);
        returns (y packed [V/2][nmass][12][Ns] complex128, per-mass stats)."""
        import torch
        nm = len(mq)
        if tuple(b.shape[-7:]) != self.spinor_shape(1)[1:]:
            raise ValueError("source has the wrong shape")
        if y is None:
            y = torch.zeros(self.packed_even_shape(nm), dtype=torch.complex128, device=b.device)
        elif tuple(y.shape) != self.packed_even_shape(nm):
            raise ValueError("y has the wrong shape")
        mqa, mqp = _f64arr(mq)
        tla, tlp = _f64arr(np.broadcast_to(np.asarray(tol, np.float64), (nm,)))
        stats = (Stats * nm)()
        st = lib().odwf_solve_masses(self._h, mqp, tlp, nm, int(inner), int(maxiter), _dev_ptr(b, "b"),
                                     _dev_ptr(y, "y"), 1 if use_y0 else 0, int(per_launch), stats,
                                     _stream(stream))
        _check(st, allow=() if raise_on_noconv else (ENOCONV, ENAN))
        return y, [s.as_dict() for s in stats]

    def deff(self, q, mq, tol=1e-12, inverse=False, inner=FP64, maxiter=100000, out=None, stream=None,
             raise_on_noconv=True):
        """odwf_deff: D_eff(m_q) q, or D_eff(m_q)^{-1} q with inverse=True, for 4D
        fields q [rhs][t][z][y][x][4][3]; returns (out, stats of the 5D solves)."""
        import torch
        nrhs = q.shape[0]
        if tuple(q.shape) != (nrhs,) + self.lattice.shape_tzyx + (4, 3):
            raise ValueError("q has the wrong shape")
        if out is None:
            out = torch.empty_like(q)
        mqa, mqp = _f64arr(np.broadcast_to(np.asarray(mq, np.float64), (nrhs,)))
        tla, tlp = _f64arr(np.broadcast_to(np.asarray(tol, np.float64), (nrhs,)))
        stats = (Stats * nrhs)()
        st = lib().odwf_deff(self._h, 1 if inverse else 0, mqp, tlp, nrhs, int(inner), int(maxiter),
                             _dev_ptr(q, "q"), _dev_ptr(out, "out"), stats, _stream(stream))
        _check(st, allow=() if raise_on_noconv else (ENOCONV, ENAN))
        return out, [s.as_dict() for s in stats]

    def force(self, chi, psi, F=None, accumulate=False, stream=None):
        """odwf_force: F_mu(x) = TA(U_mu(x) M_mu(x)) of Re <chi, W psi>; chi, psi
        [Ns][t][z][y][x][4][3] (or [1][...]) device fields; returns F
        [t][z][y][x][4][3][3] complex128 (added to F when accumulate)."""
        import torch
        for v, nm in ((chi, "chi"), (psi, "psi")):
            if tuple(v.shape[-7:]) != self.spinor_shape(1)[1:] or v.numel() != int(np.prod(self.spinor_shape(1))):
                raise ValueError(f"{nm} has the wrong shape")
        if F is None:
            F = torch.zeros(self.lattice.shape_tzyx + (4, 3, 3), dtype=torch.complex128, device=chi.device)
        _check(lib().odwf_force(self._h, _dev_ptr(chi, "chi"), _dev_ptr(psi, "psi"), 1 if accumulate else 0,
                                _dev_ptr(F, "F"), _stream(stream)))
        return F

    def reserve(self, nrhs, inner, stream=None):
        """Allocate the workspaces of a solve of nrhs right-hand sides now."""
        _check(lib().odwf_solver_reserve(self._h, int(nrhs), int(inner), _stream(stream)))

    def close(self):
        if self._h:
            lib().odwf_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Continuous-batching engine over one solver (see odwf_batch_* in odwf.h)."""

    def __init__(self, solver, max_slots, inner=FP32):
        self.solver = solver
        self.max_slots = int(max_slots)
        h = _vp()
        _check(lib().odwf_batch_create(solver._h, self.max_slots, int(inner), ctypes.byref(h)))
        self._h = h

    def admit(self, b, mq, tol, maxiter=100000, stream=None):
        """Admit one right-hand side b[Ns][t][z][y][x][4][3]; returns the slot or
        None when no slot is free."""
        slot = ctypes.c_int(-1)
        st = lib().odwf_batch_admit(self._h, _dev_ptr(b, "b"), float(mq), float(tol), int(maxiter),
                                    ctypes.byref(slot), _stream(stream))
        if st == EBUSY:
            return None
        _check(st)
        return slot.value

    def step(self, iters, stream=None):
        _check(lib().odwf_batch_step(self._h, int(iters), _stream(stream)))

    def poll(self, slot, stream=None):
        done = ctypes.c_int()
        s = Stats()
        _check(lib().odwf_batch_poll(self._h, int(slot), ctypes.byref(done), ctypes.byref(s),
                                     _stream(stream)))
        return bool(done.value), s.as_dict()

    def retire(self, slot, x, stream=None):
        s = Stats()
        _check(lib().odwf_batch_retire(self._h, int(slot), _dev_ptr(x, "x"), ctypes.byref(s),
                                       _stream(stream)))
        return s.as_dict()

    def free_slots(self):
        n = ctypes.c_int()
        _check(lib().odwf_batch_free_slots(self._h, ctypes.byref(n)))
        return n.value

    def nbytes(self):
        """Device bytes the engine holds."""
        b = ctypes.c_size_t()
        _check(lib().odwf_batch_bytes(self._h, ctypes.byref(b)))
        return b.value

    def close(self):
        if self._h:
            lib().odwf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
