/*
 * odwf.h - C ABI of libodwf.so, the MI355X (gfx950) library for the even-odd
 * preconditioned optimal domain-wall fermion (ODWF) operator and the
 * conjugate-gradient solves on its normal operator.
 *
 * Paper: T.-W. Chiu, "Simulation of dynamical (u,d,s,c) domain-wall/overlap
 * quarks at the physical point", LATTICE2018, arXiv:1811.08095.
 *
 * Operator (§2: optimal domain-wall fermion with c = 1, d = 0, H = H_w,
 * m_PV = 2 m0, R5-symmetric weights omega_s):
 *     D(m_q) = omega D_w (1 + L) + (1 - L),   L = P_- L_- + P_+ L_+,
 *     (L_+ psi)_s = psi_{s-1}, (L_+ psi)_1 = -mu psi_{Ns},
 *     (L_- psi)_s = psi_{s+1}, (L_- psi)_{Ns} = -mu psi_1,   mu = m_q / (2 m0),
 *     (D_w psi)(x) = (4 - m0) psi(x) - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                    + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)],
 * hops across the t boundary multiplied by bc_t.  Even-odd form (not in the
 * paper; the standard Schur complement on even sites, unit-diagonal form):
 *     W = D_w - (4 - m0),  A = (4 - m0) + omega^{-1} (1 - L)(1 + L)^{-1},
 *     S_e = 1 - A^{-1} W_eo A^{-1} W_oe, and conjugate gradient on S_e^dag S_e (§2).
 *
 * Conventions shared by every entry point
 *   - gamma matrices: chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 *     gamma_4 = [[0, 1], [1, 0]], gamma5 = diag(1, 1, -1, -1).
 *   - dims[4] = {Lx, Ly, Lz, Lt}; every extent even and >= 2.  Site order: x
 *     fastest, then y, z, t.  Parity (x + y + z + t) mod 2, 0 = even.
 *   - Canonical gauge field: complex128 [t][z][y][x][mu = x, y, z, t][3][3],
 *     row-major 3x3, U_mu(x) links x to x + mu; links must be SU(3) (det 1)
 *     for the 12-real compressed copies used by the reduced-precision paths.
 *   - Canonical spinor field: complex128 [rhs][s][t][z][y][x][spin 4][color 3],
 *     always on the device.  Ns must be one of 4, 8, 16, 32.
 *   - Ownership: the caller owns every in / out / b / x buffer and keeps it
 *     valid until the work queued on `stream` has finished; the library owns
 *     its resident gauge copies, packed layouts and workspaces.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *     Calls return once the work is queued, except odwf_solve and the batch
 *     poll/retire calls, which synchronise with `stream`.
 *   - Errors: every call returns an odwf_status; no exception or abort crosses
 *     the ABI; odwf_last_error() gives a thread-local message for the last
 *     failing call of the calling thread.
 *   - Threads: handles are immutable after creation except batches.  Calls on
 *     one solver from several threads are serialised by a lock; the solver
 *     keeps its workspaces per stream, so calls on different streams never
 *     share a buffer.  A batch is used from one thread at a time.
 *   - Tuning (environment, read at every hopping-kernel launch; results do not
 *     depend on them beyond rounding order of the partial sums):
 *       ODWF_TRAVERSAL = "linear" | "xcd" | "Ty,Tz" | "Ty,Tz,Tt" | "Ty,Tz,Tt,Tx"
 *         block order of the hopping kernel.  Default, when the x half-rows
 *         split into whole blocks: tiles of one x-row segment by 8 x 4 (y, z)
 *         rows (4 x 4 when Ly is not a multiple of 8) walked with t innermost;
 *         Tt > 0 cuts t into chunks of Tt, Tx is the number of x-row segments
 *         per tile (0: the whole row).  Otherwise XCD-aware contiguous ranges;
 *       ODWF_XCD = "contiguous" | "lockstep" | "lockstep:Gy"  how the eight
 *         XCDs share the tiles: contiguous runs of tiles, or (default) groups
 *         of Gy x 8/Gy adjacent tiles walked by the eight XCDs in lockstep.
 */
#ifndef ODWF_H
#define ODWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct odwf_lattice_s* odwf_lattice;
typedef struct odwf_solver_s* odwf_solver;
typedef struct odwf_batch_s* odwf_batch;

typedef enum {
  ODWF_OK = 0,
  ODWF_EINVAL = -1,  /* bad argument: null pointer, bad extent, unsupported Ns ... */
  ODWF_ENOMEM = -2,  /* device allocation failed or admission budget exceeded      */
  ODWF_EHIP = -3,    /* a HIP runtime call failed                                   */
  ODWF_ENOCONV = -4, /* solver reached maxiter; x holds the best iterate            */
  ODWF_ENAN = -5,    /* NaN/Inf met in a residual norm                              */
  ODWF_EBUSY = -6    /* batch has no free slot                                      */
} odwf_status;

/* Precision of the spinor storage / arithmetic of an apply or of the inner
 * solver.  FP64: double spinors, double 18-real links.  FP32: float spinors,
 * float 12-real links (third row rebuilt in the kernel).  FP16S / BF16S:
 * half / bfloat16 spinors with one float scale per 5D site (site, s, rhs),
 * float 12-real links, float arithmetic. */
typedef enum { ODWF_FP64 = 0, ODWF_FP32 = 1, ODWF_FP16S = 2, ODWF_BF16S = 3 } odwf_prec;

/* Operators of odwf_apply, on full-lattice canonical fields.  Where an operator
 * produces only even (odd) sites the other parity of `out` is written as zero.
 *   HOP_EO:       out_e = W_eo in_o                (W = D_w - (4 - m0))
 *   HOP_OE:       out_o = W_oe in_e
 *   M5INV:        out   = A^{-1} in               (every site)
 *   D, DDAG:      out   = D in, D^dag in
 *   DDAGD:        out   = D^dag D in
 *   SCHUR:        out_e = S_e in_e
 *   SCHUR_DAG:    out_e = S_e^dag in_e
 *   SCHUR_NORMAL: out_e = S_e^dag S_e in_e */
typedef enum {
  ODWF_OP_HOP_EO = 0,
  ODWF_OP_HOP_OE = 1,
  ODWF_OP_M5INV = 2,
  ODWF_OP_D = 3,
  ODWF_OP_DDAG = 4,
  ODWF_OP_DDAGD = 5,
  ODWF_OP_SCHUR = 6,
  ODWF_OP_SCHUR_DAG = 7,
  ODWF_OP_SCHUR_NORMAL = 8
} odwf_op;

/* EO_NORMAL: solve S_e^dag S_e y = b_e (even sites of b); x_e = y, x_o = 0.
 * FULL:      solve D x = b: b' = omega^{-1} b,
 *            phi_e = A^{-1}(b'_e - W_eo A^{-1} b'_o),
 *            CG on S_e^dag S_e y_e = S_e^dag phi_e,
 *            y_o = A^{-1}(b'_o - W_oe y_e),  x = (1 + L)^{-1} y.
 * The stopping test is on the system CG iterates: |f - S_e^dag S_e y| <= tol |f|. */
typedef enum { ODWF_SOLVE_EO_NORMAL = 0, ODWF_SOLVE_FULL = 1 } odwf_mode;

typedef struct {
  int iters;             /* CG iterations (inner iterations for mixed solves)          */
  int reliable_updates;  /* FP32 inner: FP64 true-residual updates of this right-hand
                            side's own iterate, the final confirmation included; else 0 */
  int outer_steps;       /* FP16S/BF16S inner: FP64 defect-correction steps this
                            right-hand side took part in; else 0                       */
  int status;            /* odwf_status of this right-hand side                        */
  double true_rel_resid; /* |f - S_e^dag S_e y| / |f|, recomputed in FP64 at the end   */
  double full_rel_resid; /* FULL mode: |b - D x| / |b| in FP64; -1 in EO_NORMAL mode   */
  double seconds;        /* wall time from the call's start until this right-hand side
                            was seen finished (the whole call for the last one)        */
} odwf_stats;

/* ---- lattices and gauge fields ----------------------------------------- */

/* Create a lattice of extents dims on HIP device `device`; bc_t = +1 or -1 is
 * the boundary factor of hops across the t boundary. */
odwf_status odwf_lattice_create(const int dims[4], int bc_t, int device, odwf_lattice* out);

/* Load (or replace) the gauge field.  U is the canonical complex128 field,
 * a device pointer when on_device != 0, else a host pointer.  The library
 * builds its resident copies (FP64 18-real and FP32 12-real, split by parity,
 * backward links stored as U_mu(x - mu)^dag); U may be freed once the work on
 * `stream` has finished. */
odwf_status odwf_lattice_load_gauge(odwf_lattice lat, const void* U, int on_device, void* stream);

/* Device bytes held by the lattice (resident gauge copies). */
odwf_status odwf_lattice_bytes(odwf_lattice lat, size_t* bytes);

void odwf_lattice_destroy(odwf_lattice lat);

/* ---- solver: operator parameters on a lattice ------------------------- */

/* Ns in {4, 8, 16, 32}; m0 the domain-wall height (paper: 1.3); omega[Ns]
 * the weights omega_s (host array, copied; all > 0).  R5 symmetry
 * (palindromic omega) is the paper's choice but is not required here. */
odwf_status odwf_solver_create(odwf_lattice lat, int Ns, double m0, const double* omega,
                               odwf_solver* out);

void odwf_solver_destroy(odwf_solver s);

/* out = op(in) for nrhs right-hand sides, each with its bare quark mass
 * mq[r] (host array; mu_r = mq[r] / (2 m0)).  in/out: device canonical
 * spinor fields of nrhs * Ns * V * 12 complex128, distinct buffers.  prec
 * selects the precision of the hopping and fifth-dimension kernels (the
 * canonical fields stay complex128). */
odwf_status odwf_apply(odwf_solver s, odwf_op op, const double* mq, odwf_prec prec, int nrhs,
                       const void* in, void* out, void* stream);

/* Bytes of the per-device scratch array behind odwf_apply_noalloc. */
#define ODWF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* odwf_apply without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operators, arguments, results and errors as odwf_apply; the
 * packed half fields it works in are carved from a file-scope device array of
 * ODWF_NOALLOC_SCRATCH_BYTES per GPU (held from the first lattice created on
 * that GPU until the process ends) instead of the solver's workspace.  A call
 * whose operator needs more scratch than that for one launch's right-hand
 * sides (at most 256 / Ns) returns ODWF_ENOMEM with the sizes in
 * odwf_last_error() and queues nothing.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads, other
 * solvers) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero.  No profiling events are recorded. */
odwf_status odwf_apply_noalloc(odwf_solver s, odwf_op op, const double* mq, odwf_prec prec,
                               int nrhs, const void* in, void* out, void* stream);

/* Solve for nrhs right-hand sides (independent masses mq[r] and tolerances
 * tol[r], host arrays).  inner = ODWF_FP64: plain FP64 CG; ODWF_FP32: FP32 CG
 * with FP64 reliable updates; ODWF_FP16S / ODWF_BF16S: FP64 defect correction
 * around an inner CG in that storage.  b, x: device canonical fields; when
 * use_x0 != 0, x holds the initial guess on entry, otherwise x is ignored on
 * entry and may alias b.  stats: host array of nrhs records (may be NULL).
 * Returns ODWF_ENOCONV if any right-hand side missed its tolerance within
 * maxiter (x then holds the last iterate), ODWF_ENAN on a NaN/Inf residual. */
odwf_status odwf_solve(odwf_solver s, odwf_mode mode, const double* mq, const double* tol,
                       int nrhs, odwf_prec inner, int maxiter, const void* b, void* x,
                       int use_x0, odwf_stats* stats, void* stream);

/* Multi-mass solves for one source (paper §2: the fermion forces of the HMC
 * need the solution of the even-odd normal system at several quark masses for
 * one pseudofermion field -- the Hasenbusch masses, m_ud, m_s, m_c, and the
 * Pauli-Villars mass 2 m0 of Eq. (1)-(2)):
 *     S_e(m_k)^dag S_e(m_k) y_k = b_e,   k = 0 .. nmass - 1,
 * all masses iterated together in multi-right-hand-side CG launches, so that
 * every link load serves all of them (per mass: own mu = mq[k] / (2 m0), own
 * tolerance tol[k], own CG scalars).  1 <= nmass <= 256 / Ns (and <= 16).
 * b: ONE canonical device field (its even sites are the source of every mass;
 * its odd sites are not read).  y: caller-owned device array in the packed
 * even-half FP64 layout of the library (nothing canonical is allocated, so
 * several masses fit where canonical outputs would not):
 *     complex128 y[((j * nmass + k) * 12 + c) * Ns + s],
 *     j = ((t * Lz + z) * Ly + y) * (Lx / 2) + x / 2 over the even sites
 *         (x + y + z + t even), c = spin * 3 + colour, s = 0 .. Ns - 1,
 * i.e. nmass * (V / 2) * Ns * 12 complex128.  With use_y0 != 0, y holds the
 * initial guesses on entry.  per_launch = masses iterated together in one
 * multi-right-hand-side CG (1 .. nmass), or 0 to let the library choose: all
 * of them together while one right-hand side's FP32 half field fits the
 * 256 MB memory-side cache, one at a time above that (where the wider sites of
 * a shared launch cost more neighbour re-fetch than its shared links save).
 * inner, maxiter, stats, stream and the return codes as for odwf_solve (mode
 * EO_NORMAL); the workspaces are those of an odwf_solve of per_launch
 * right-hand sides (plus one packed field of per_launch masses when
 * per_launch < nmass). */
odwf_status odwf_solve_masses(odwf_solver s, const double* mq, const double* tol, int nmass,
                              odwf_prec inner, int maxiter, const void* b, void* y, int use_y0,
                              int per_launch, odwf_stats* stats, void* stream);

/* Effective 4D operator (paper §2: the effective 4D operator of the optimal
 * domain-wall fermion is exactly the shifted Zolotarev optimal rational
 * approximation of the overlap operator; with the Pauli-Villars normalisation
 * of Eq. (1)-(2)):
 *     D_eff(m_q) = (1 + mu)/2 + (1 - mu)/2 gamma5 S(H_w),   mu = m_q / (2 m0),
 *     S(H) = (1 - prod_s T_s)(1 + prod_s T_s)^{-1},  T_s = (1 - w_s H)(1 + w_s H)^{-1},
 * computed through the 5D operator with R taking the chirality-plus spins of
 * slice Ns and the chirality-minus spins of slice 1 (the slices the m_q
 * boundary term couples), R^T its embedding:
 *     inverse == 0:  out = D_eff(m_q) q      = R D(m_PV)^{-1} D(m_q) R^T q,
 *     inverse != 0:  out = D_eff(m_q)^{-1} q = R D(m_q)^{-1} D(m_PV) R^T q
 *                    (the 4D quark propagator),  m_PV = 2 m0;
 * one FULL odwf_solve per right-hand side (tolerance tol[r], inner precision,
 * maxiter, stats as there; apply: the solve is at m_PV, propagator: at
 * m_q[r]).  q, out: device canonical 4D spinor fields complex128
 * [rhs][t][z][y][x][spin 4][color 3], distinct.  Workspaces: two canonical 5D
 * fields of one launch's right-hand sides plus those of the solve.  Returns as
 * odwf_solve; synchronises with `stream`. */
odwf_status odwf_deff(odwf_solver s, int inverse, const double* mq, const double* tol, int nrhs,
                      odwf_prec inner, int maxiter, const void* q, void* out, odwf_stats* stats,
                      void* stream);

/* Fermion-force primitive (paper §2: the forces of the HMC's fermion actions
 * differentiate bilinears of the hopping term with the solutions of the
 * normal equations).  For
 *     S = Re <chi, W psi> = Re sum_s sum_x chi(x, s)^dag (W psi)(x, s),
 * W the hopping term of D_w (the header's D_w without its 4 - m0 diagonal,
 * hops across the t boundary times bc_t), every link U_mu(x) enters S only as
 *     Re tr(U_mu(x) M_mu(x)),   M = -1/2 b (A + B^dag),
 *     A = sum_{s,spin} [(1 - gamma_mu) psi(x + mu, s)] (x) chi(x, s)^dag,
 *     B = sum_{s,spin} [(1 + gamma_mu) psi(x, s)] (x) chi(x + mu, s)^dag,
 * (b = bc_t if x + mu wraps in t, else 1), and the force is
 *     F_mu(x) = TA(U_mu(x) M_mu(x)),  TA(X) = (X - X^dag)/2 - tr(X - X^dag)/6,
 * traceless anti-Hermitian, so that dS/d eps = i tr(T F_mu(x)) for
 * U_mu(x) -> exp(i eps T) U_mu(x) with T Hermitian and traceless.
 * chi, psi: device canonical spinor fields of ONE right-hand side (Ns * V * 12
 * complex128); F: device complex128 [t][z][y][x][mu][3][3], overwritten, or
 * added to when accumulate != 0 (sums of several bilinears).  FP64. */
odwf_status odwf_force(odwf_solver s, const void* chi, const void* psi, int accumulate, void* F,
                       void* stream);

/* Allocate now the workspaces odwf_solve uses on `stream` for nrhs right-hand
 * sides (at most one launch's worth, 256 / Ns, is held) in precision `inner`,
 * so that a later solve does no device allocation of its own.  Workspaces are
 * kept per stream until the solver is destroyed.  ODWF_ENOMEM if they do not
 * fit. */
odwf_status odwf_solver_reserve(odwf_solver s, int nrhs, odwf_prec inner, void* stream);

/* Device bytes odwf_solve needs beyond the resident gauge copies for a
 * lattice of extents dims (workspace only; the caller's b and x excluded). */
odwf_status odwf_footprint(const int dims[4], int Ns, int nrhs, odwf_prec inner, size_t* bytes);

/* Optimal weights (paper §2): omega_k = dn((2k - 1) K' / Ns; kappa') / lambda_min,
 * kappa'^2 = 1 - lambda_min^2 / lambda_max^2, k = 1 .. Ns/2, descending, then
 * mirrored (R5 symmetry).  Host computation; omega is a host array of Ns. */
odwf_status odwf_zolotarev_omega(int Ns, double lambda_min, double lambda_max, double* omega);

/* ---- serving: continuous batching at CG-iteration granularity ---------- */

/* A batch engine holds max_slots right-hand-side slots of one solver, solved
 * together by multi-right-hand-side CG iterations (one link load serves all
 * slots) in precision `inner` (FP64, or FP32 with FP64 reliable updates).
 * Every slot has its own mass, tolerance and CG scalars; a slot's arithmetic
 * never depends on which other slots are occupied. */
odwf_status odwf_batch_create(odwf_solver s, int max_slots, odwf_prec inner, odwf_batch* out);

/* Admit one right-hand side b (device canonical field of Ns * V * 12
 * complex128, FULL mode) with mass mq and tolerance tol into a free slot;
 * *slot receives its index.  ODWF_EBUSY when no slot is free.  b is read on
 * `stream` before the call returns to the queue. */
odwf_status odwf_batch_admit(odwf_batch bt, const void* b, double mq, double tol, int maxiter,
                             int* slot, void* stream);

/* Run `iters` CG iterations on every active slot (inactive slots are left
 * untouched). */
odwf_status odwf_batch_step(odwf_batch bt, int iters, void* stream);

/* *done = 1 when the slot has converged, hit maxiter or failed. */
odwf_status odwf_batch_poll(odwf_batch bt, int slot, int* done, odwf_stats* stats, void* stream);

/* Finish a slot: FP64 true residual, reconstruction of x (device canonical
 * field of Ns * V * 12 complex128), and release of the slot. */
odwf_status odwf_batch_retire(odwf_batch bt, int slot, void* x, odwf_stats* stats, void* stream);

/* Slots currently free. */
odwf_status odwf_batch_free_slots(odwf_batch bt, int* n);

/* Device bytes odwf_batch_create allocates for an engine of max_slots slots
 * on a lattice of extents dims (host computation; the resident lattice and
 * solver excluded), so that a server can admit engines by HBM footprint
 * before creating them. */
odwf_status odwf_batch_footprint(const int dims[4], int Ns, int max_slots, odwf_prec inner,
                                 size_t* bytes);

/* Device bytes an existing engine holds (equal to its odwf_batch_footprint). */
odwf_status odwf_batch_bytes(odwf_batch bt, size_t* bytes);

void odwf_batch_destroy(odwf_batch bt);

/* ---- profiling --------------------------------------------------------- */

/* Kernel-time accounting with HIP events recorded on the launching stream
 * around every hopping-kernel launch.  enable != 0 turns it on (and clears the
 * counters).  odwf_profile_read synchronises the recorded events and returns
 * the number of hopping launches, their summed duration in milliseconds and
 * their summed algorithmic bytes (spinor reads and writes plus link reads,
 * plus the vector streams a launch carries for a fused CG step).  Batch-engine
 * launches restricted to the active slots count with the bytes of every slot
 * (exact while all slots are active); the batch's FP64 reliable-update
 * launches, which run only for slots that requested an update, are not
 * counted. */
odwf_status odwf_profile_enable(int enable);
odwf_status odwf_profile_read(long long* launches, double* ms, double* bytes);

/* The same counters restricted to one instantiation of the hopping kernel:
 * storage precision `prec` and dag = 0 (W, forward projector 1 - gamma) or
 * dag = 1 (W^dag). */
odwf_status odwf_profile_read_kernel(odwf_prec prec, int dag, long long* launches, double* ms,
                                     double* bytes);

/* Thread-local message describing the last error of the calling thread. */
const char* odwf_last_error(void);

/* Library version string. */
const char* odwf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ODWF_H */
