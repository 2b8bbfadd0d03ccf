// Batch engine: continuous batching of CG solves at iteration granularity.
//
// An engine owns max_slots right-hand-side slots of one solver (one lattice,
// one Ns).  All slots advance together through multi-right-hand-side CG
// iterations on S_e^dag S_e (one link load per site serves every slot), but
// each slot has its own mass (corner factor -mu of the fifth-dimension
// matrices), tolerance, iteration cap and CG scalars.  Every per-slot decision
// is taken on the device from that slot's own scalars, in the iteration where
// it arises: the FP32 / FP64 iterate advances while the slot is active; when
// its iterated residual drops below delta * max|r| (FP32 inner), meets the
// tolerance or reaches the cap, the same iteration runs a gated FP64 update
// for exactly those slots (y += x_s, r = f - N y with the FP64 operator) and
// the true residual decides convergence.  Kernels skip the lanes of inactive
// slots.  A slot's arithmetic is therefore identical whichever other slots are
// occupied, and the host only enqueues work and polls flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"
#include "solver.h"

using namespace odwf;

struct odwf_batch_s {
  odwf_solver S = nullptr;
  int k = 0;          // slots
  int inner = PREC32; // inner precision
  Workspace ws;       // engine-owned buffers
  // k-slot fields
  HV f, y, e2, o0, bo;          // FP64: rhs, solution, scratch even/odd, omega^{-1} b (odd)
  HV p, r, x, t, v;             // inner precision (x unused for FP64: y accumulates)
  // single right-hand-side scratch (FP64) for admission and retirement
  HV s_e0, s_e1, s_e2, s_o0, s_bo;
  CGScal* dscal = nullptr;
  double* partial = nullptr;
  double* dres = nullptr;
  CGScal* hscal = nullptr;      // pinned mirror of dscal
  bool cache_valid = false;
  std::vector<int> used;
  std::vector<double> mq;
  std::vector<std::chrono::steady_clock::time_point> t_admit;
};

#define BCHK(expr)                                                                       \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      set_error(std::string("batch: HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return ODWF_EHIP;                                                                  \
    }                                                                                    \
  } while (0)

#define BREQ(cond, msg)   \
  do {                    \
    if (!(cond)) {        \
      set_error(msg);     \
      return ODWF_EINVAL; \
    }                     \
  } while (0)

static OpCtx ctx_of(odwf_batch B, hipStream_t st, int prec, int nrhs, const double* kappa) {
  OpCtx c;
  c.S = B->S;
  c.st = st;
  c.prec = prec;
  c.nrhs = nrhs;
  for (int q = 0; q < MAXRHS; q++) c.kappa[q] = q < nrhs ? kappa[q] : 0.0;
  return c;
}

static void kappas(odwf_batch B, double* kap) {
  for (int q = 0; q < MAXRHS; q++) kap[q] = q < B->k ? -B->mq[q] / (2.0 * B->S->m0) : 0.0;
}

// device bytes a batch engine allocates (the buffers of odwf_batch_create)
static size_t batch_footprint_bytes(long h, int Ns, int k, int inner) {
  auto buf = [](size_t b) { return b ? b : size_t(16); };
  size_t t = 5 * buf(half_bytes(h, k, Ns, PREC64));  // f, y, e2, o0, bo
  const int ninner = inner == PREC64 ? 4 : 5;       // p, r, t, v (+ x)
  t += ninner * buf(half_bytes(h, k, Ns, inner));
  if (k > 1) t += 5 * buf(half_bytes(h, 1, Ns, PREC64));  // admission / retirement scratch
  const int nb = std::max(hop_nblocks((int)h, k, Ns), vec_nblocks(h, k, Ns));
  t += partial_bytes(nb, k) + MAXRHS * sizeof(CGScal) + 4 * MAXRHS * sizeof(double);
  return t;
}

extern "C" odwf_status odwf_batch_footprint(const int dims[4], int Ns, int max_slots, odwf_prec inner,
                                            size_t* bytes) {
  BREQ(dims && bytes, "odwf_batch_footprint: null argument");
  BREQ(Ns == 4 || Ns == 8 || Ns == 16 || Ns == 32, "odwf_batch_footprint: unsupported Ns");
  BREQ(max_slots >= 1 && max_slots <= max_rhs_per_launch(Ns), "odwf_batch_footprint: bad max_slots");
  BREQ(inner == ODWF_FP64 || inner == ODWF_FP32, "odwf_batch_footprint: inner must be FP64 or FP32");
  for (int d = 0; d < 4; d++) BREQ(dims[d] >= 2 && dims[d] % 2 == 0, "odwf_batch_footprint: bad extent");
  const long h = (long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
  *bytes = batch_footprint_bytes(h, Ns, max_slots, (int)inner);
  return ODWF_OK;
}

extern "C" odwf_status odwf_batch_bytes(odwf_batch B, size_t* bytes) {
  BREQ(B && bytes, "odwf_batch_bytes: null argument");
  *bytes = B->ws.total();
  return ODWF_OK;
}

extern "C" odwf_status odwf_batch_create(odwf_solver S, int max_slots, odwf_prec inner,
                                         odwf_batch* out) {
  BREQ(S && out, "odwf_batch_create: null argument");
  BREQ(S->lat->loaded, "odwf_batch_create: gauge field not loaded");
  BREQ(max_slots >= 1 && max_slots <= max_rhs_per_launch(S->Ns),
       "odwf_batch_create: max_slots must be in [1, 256 / Ns] and <= 16");
  BREQ(inner == ODWF_FP64 || inner == ODWF_FP32, "odwf_batch_create: inner must be FP64 or FP32");
  BCHK(hipSetDevice(S->lat->device));
  odwf_batch B = new odwf_batch_s();
  B->S = S;
  B->k = max_slots;
  B->inner = inner;
  const long h = S->lat->g.h;
  const int Ns = S->Ns, k = max_slots;
  Workspace& W = B->ws;
  B->f = W.half("f", h, k, Ns, PREC64);
  B->y = W.half("y", h, k, Ns, PREC64);
  B->e2 = W.half("e2", h, k, Ns, PREC64);
  B->o0 = W.half("o0", h, k, Ns, PREC64);
  B->bo = W.half("bo", h, k, Ns, PREC64);
  B->p = W.half("p", h, k, Ns, inner);
  B->r = W.half("r", h, k, Ns, inner);
  B->t = W.half("t", h, k, Ns, inner);
  B->v = W.half("v", h, k, Ns, inner);
  if ((int)inner != PREC64) B->x = W.half("x", h, k, Ns, inner);
  if (k == 1) {
    // one slot: admission and retirement work in the slot's own fields (same
    // layout); every step of both sequences reads and writes them in an order
    // in which no value is overwritten before its last use
    B->s_e0 = B->f;
    B->s_e1 = B->y;
    B->s_e2 = B->e2;
    B->s_o0 = B->o0;
    B->s_bo = B->bo;
  } else {
    B->s_e0 = W.half("s_e0", h, 1, Ns, PREC64);
    B->s_e1 = W.half("s_e1", h, 1, Ns, PREC64);
    B->s_e2 = W.half("s_e2", h, 1, Ns, PREC64);
    B->s_o0 = W.half("s_o0", h, 1, Ns, PREC64);
    B->s_bo = W.half("s_bo", h, 1, Ns, PREC64);
  }
  const int nb = std::max(hop_nblocks((int)h, k, Ns), vec_nblocks(h, k, Ns));
  B->partial = (double*)W.get("partial", partial_bytes(nb, k));
  B->dscal = (CGScal*)W.get("scal", MAXRHS * sizeof(CGScal));
  B->dres = (double*)W.get("res", 4 * MAXRHS * sizeof(double));
  bool ok = B->f.d && B->y.d && B->e2.d && B->o0.d && B->bo.d && B->p.d && B->r.d && B->t.d &&
            B->v.d && ((int)inner == PREC64 || B->x.d) && B->s_e0.d && B->s_e1.d && B->s_e2.d &&
            B->s_o0.d && B->s_bo.d && B->partial && B->dscal && B->dres;
  if (ok && hipHostMalloc((void**)&B->hscal, MAXRHS * sizeof(CGScal), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    B->hscal = nullptr;
    ok = false;
  }
  if (!ok) {
    delete B;
    set_error("odwf_batch_create: out of device memory");
    return ODWF_ENOMEM;
  }
  std::vector<CGScal> z(MAXRHS);
  std::memset(z.data(), 0, z.size() * sizeof(CGScal));
  BCHK(hipMemcpy(B->dscal, z.data(), z.size() * sizeof(CGScal), hipMemcpyHostToDevice));
  std::memcpy(B->hscal, z.data(), z.size() * sizeof(CGScal));
  B->cache_valid = true;
  B->used.assign(k, 0);
  B->mq.assign(k, 0.0);
  B->t_admit.resize(k);
  *out = B;
  return ODWF_OK;
}

extern "C" odwf_status odwf_batch_free_slots(odwf_batch B, int* n) {
  BREQ(B && n, "odwf_batch_free_slots: null argument");
  *n = (int)std::count(B->used.begin(), B->used.end(), 0);
  return ODWF_OK;
}

extern "C" odwf_status odwf_batch_admit(odwf_batch B, const void* b, double mq, double tol,
                                        int maxiter, int* slot, void* stream) {
  BREQ(B && b && slot, "odwf_batch_admit: null argument");
  BREQ(std::isfinite(mq) && tol > 0 && tol < 1 && maxiter >= 1, "odwf_batch_admit: bad mq, tol or maxiter");
  int q = -1;
  for (int i = 0; i < B->k; i++)
    if (!B->used[i]) {
      q = i;
      break;
    }
  if (q < 0) {
    set_error("odwf_batch_admit: no free slot");
    return ODWF_EBUSY;
  }
  BCHK(hipSetDevice(B->S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  odwf_solver S = B->S;
  const Geom& g = S->lat->g;
  const long h = g.h;
  const int Ns = S->Ns;
  double kap1[MAXRHS] = {-mq / (2.0 * S->m0)};
  OpCtx c1 = ctx_of(B, st, PREC64, 1, kap1);
  // f = S_e^dag phi_e,  phi_e = A^{-1}(b'_e - W_eo A^{-1} b'_o),  b' = omega^{-1} b
  BCHK(launch_pack_spinor(PREC64, b, 0, B->s_e2.d, nullptr, 0, 1, Ns, g, st));
  BCHK(launch_pack_spinor(PREC64, b, 0, B->s_bo.d, nullptr, 1, 1, Ns, g, st));
  BCHK(m5(c1, B->s_e2, B->s_e2, prog_omega_inv()));
  BCHK(m5(c1, B->s_bo, B->s_bo, prog_omega_inv()));
  BCHK(m5(c1, B->s_bo, B->s_o0, prog_ainv()));
  HopOpt kp;
  kp.x = &B->s_e2;
  kp.ch = -1.0;
  kp.cx = 1.0;
  kp.po = prog_ainv();
  BCHK(hop(c1, 0, 0, B->s_o0, &B->s_e1, kp));
  BCHK(apply_schur_dag(c1, B->s_e1, B->s_e2, B->s_o0, B->s_e0));
  // scatter into the slot (a one-slot engine prepared f and bo in place)
  if (B->s_e0.d != B->f.d)
    BCHK(launch_vec_copy_rhs(PREC64, B->s_e0.d, nullptr, 1, 0, PREC64, B->f.d, nullptr, B->k, q, h, Ns, st));
  BCHK(launch_vec_copy_rhs(PREC64, nullptr, nullptr, 1, 0, PREC64, B->y.d, nullptr, B->k, q, h, Ns, st));
  if (B->s_bo.d != B->bo.d)
    BCHK(launch_vec_copy_rhs(PREC64, B->s_bo.d, nullptr, 1, 0, PREC64, B->bo.d, nullptr, B->k, q, h, Ns, st));
  BCHK(launch_vec_copy_rhs(PREC64, B->s_e0.d, nullptr, 1, 0, B->inner, B->r.d, B->r.sc, B->k, q, h, Ns, st));
  BCHK(launch_vec_copy_rhs(PREC64, B->s_e0.d, nullptr, 1, 0, B->inner, B->p.d, B->p.sc, B->k, q, h, Ns, st));
  if (B->inner != PREC64)
    BCHK(launch_vec_copy_rhs(PREC64, nullptr, nullptr, 1, 0, B->inner, B->x.d, B->x.sc, B->k, q, h, Ns, st));
  // |f|^2
  int nbv = 0;
  BCHK(launch_vec_norm2(PREC64, B->s_e0.d, nullptr, B->partial, h, 1, Ns, &nbv, st));
  BCHK(launch_fin(FIN_SUM, B->partial, nbv, 1, nullptr, B->dres, st));
  double f2 = 0.0;
  BCHK(hipMemcpyAsync(&f2, B->dres, sizeof(double), hipMemcpyDeviceToHost, st));
  BCHK(hipStreamSynchronize(st));
  CGScal c;
  std::memset(&c, 0, sizeof(c));
  c.f2 = f2;
  c.rr = f2;
  c.rmax2 = f2;
  c.tol2 = tol * tol;
  c.maxiter = maxiter;
  c.confirm = 1;
  c.delta2 = B->inner == PREC64 ? 0.0 : RELIABLE_DELTA2;
  if (!std::isfinite(f2)) {
    c.nan = 1;
  } else if (f2 == 0.0) {
    c.converged = 1;
  } else {
    c.active = 1;
  }
  BCHK(hipMemcpyAsync(B->dscal + q, &c, sizeof(c), hipMemcpyHostToDevice, st));
  BCHK(hipStreamSynchronize(st));
  B->used[q] = 1;
  B->mq[q] = mq;
  B->t_admit[q] = std::chrono::steady_clock::now();
  B->cache_valid = false;
  *slot = q;
  return ODWF_OK;
}

// one iteration for every active slot, followed by the gated FP64 update of
// the slots that asked for one in this iteration
static hipError_t batch_iteration(odwf_batch B, hipStream_t st) {
  odwf_solver S = B->S;
  const long h = S->lat->g.h;
  const int Ns = S->Ns, k = B->k;
  double kap[MAXRHS];
  kappas(B, kap);
  OpCtx cin = ctx_of(B, st, B->inner, k, kap);
  OpCtx c64 = ctx_of(B, st, PREC64, k, kap);
  const int nbh = hop_nblocks((int)h, k, Ns);
  HV* xacc = B->inner == PREC64 ? &B->y : &B->x;
  HopOpt k4;
  k4.cg_r = &B->r;
  k4.scal = B->dscal;
  k4.partial = B->partial;
  HIPRET(apply_normal(cin, B->p, B->t, B->v, B->v, B->partial, &k4, B->dscal, GATE_ACTIVE));
  HIPRET(launch_fin(FIN_BETA, B->partial, nbh, k, B->dscal, nullptr, st));
  HIPRET(launch_vec_cg_step(B->inner, B->r.d, B->r.sc, B->p.d, B->p.sc, xacc->d, xacc->sc, B->dscal, h, k,
                            Ns, st));
  // gated update: y += x_s, x_s = 0, r = f - N y (FP64), true |r|^2
  if (B->inner != PREC64) {
    HIPRET(launch_vec_convert(B->inner, B->x.d, B->x.sc, PREC64, B->y.d, nullptr, 1, h, k, Ns, st,
                              B->dscal, GATE_UPDATE));
    HIPRET(launch_vec_zero(B->inner, B->x.d, B->x.sc, h, k, Ns, st, B->dscal, GATE_UPDATE));
  }
  HopOpt kr;
  kr.partial = B->partial;
  kr.cg_p = &B->f;
  HIPRET(apply_normal(c64, B->y, B->o0, B->e2, B->e2, nullptr, &kr, B->dscal, GATE_UPDATE));
  HIPRET(launch_vec_convert(PREC64, B->e2.d, nullptr, B->inner, B->r.d, B->r.sc, 0, h, k, Ns, st,
                            B->dscal, GATE_UPDATE));
  return launch_fin(FIN_INIT, B->partial, nbh, k, B->dscal, nullptr, st, 1);
}

extern "C" odwf_status odwf_batch_step(odwf_batch B, int iters, void* stream) {
  BREQ(B && iters >= 0, "odwf_batch_step: bad argument");
  BCHK(hipSetDevice(B->S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (std::count(B->used.begin(), B->used.end(), 1) == 0) return ODWF_OK;
  for (int i = 0; i < iters; i++) BCHK(batch_iteration(B, st));
  B->cache_valid = false;
  return ODWF_OK;
}

static odwf_status refresh(odwf_batch B, hipStream_t st) {
  if (B->cache_valid) return ODWF_OK;
  BCHK(hipMemcpyAsync(B->hscal, B->dscal, B->k * sizeof(CGScal), hipMemcpyDeviceToHost, st));
  BCHK(hipStreamSynchronize(st));
  B->cache_valid = true;
  return ODWF_OK;
}

static void fill_stats(odwf_batch B, int q, odwf_stats* s) {
  const CGScal& c = B->hscal[q];
  s->iters = c.iters;
  s->reliable_updates = c.nupd;
  s->outer_steps = 0;
  s->status = c.nan ? ODWF_ENAN : (c.converged ? ODWF_OK : ODWF_ENOCONV);
  s->true_rel_resid = c.f2 > 0 ? std::sqrt(c.rr / c.f2) : 0.0;
  s->full_rel_resid = -1.0;
  s->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - B->t_admit[q]).count();
}

extern "C" odwf_status odwf_batch_poll(odwf_batch B, int slot, int* done, odwf_stats* stats,
                                       void* stream) {
  BREQ(B && done, "odwf_batch_poll: null argument");
  BREQ(slot >= 0 && slot < B->k && B->used[slot], "odwf_batch_poll: slot not in use");
  odwf_status s = refresh(B, reinterpret_cast<hipStream_t>(stream));
  if (s != ODWF_OK) return s;
  const CGScal& c = B->hscal[slot];
  *done = (!c.active && !c.update) ? 1 : 0;
  if (stats) fill_stats(B, slot, stats);
  return ODWF_OK;
}

extern "C" odwf_status odwf_batch_retire(odwf_batch B, int slot, void* x, odwf_stats* stats,
                                         void* stream) {
  BREQ(B && x, "odwf_batch_retire: null argument");
  BREQ(slot >= 0 && slot < B->k && B->used[slot], "odwf_batch_retire: slot not in use");
  BCHK(hipSetDevice(B->S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  odwf_status s0 = refresh(B, st);
  if (s0 != ODWF_OK) return s0;
  if (stats) fill_stats(B, slot, stats);
  odwf_solver S = B->S;
  const Geom& g = S->lat->g;
  const long h = g.h;
  const int Ns = S->Ns;
  double kap1[MAXRHS] = {-B->mq[slot] / (2.0 * S->m0)};
  OpCtx c1 = ctx_of(B, st, PREC64, 1, kap1);
  if (B->s_e1.d != B->y.d)
    BCHK(launch_vec_copy_rhs(PREC64, B->y.d, nullptr, B->k, slot, PREC64, B->s_e1.d, nullptr, 1, 0, h, Ns, st));
  if (B->s_bo.d != B->bo.d)
    BCHK(launch_vec_copy_rhs(PREC64, B->bo.d, nullptr, B->k, slot, PREC64, B->s_bo.d, nullptr, 1, 0, h, Ns, st));
  // y_o = A^{-1}(b'_o - W_oe y_e), x = (1 + L)^{-1} y
  HopOpt kr;
  kr.x = &B->s_bo;
  kr.ch = -1.0;
  kr.cx = 1.0;
  kr.po = prog_ainv();
  BCHK(hop(c1, 1, 0, B->s_e1, &B->s_bo, kr));
  BCHK(m5(c1, B->s_e1, B->s_e1, prog_1pl_inv()));
  BCHK(m5(c1, B->s_bo, B->s_bo, prog_1pl_inv()));
  BCHK(launch_unpack_spinor(PREC64, B->s_e1.d, nullptr, x, 0, 0, 1, Ns, g, st));
  BCHK(launch_unpack_spinor(PREC64, B->s_bo.d, nullptr, x, 0, 1, 1, Ns, g, st));
  // release the slot: inactive, no update pending
  CGScal z;
  std::memset(&z, 0, sizeof(z));
  BCHK(hipMemcpyAsync(B->dscal + slot, &z, sizeof(z), hipMemcpyHostToDevice, st));
  BCHK(hipStreamSynchronize(st));
  B->hscal[slot] = z;
  B->used[slot] = 0;
  return ODWF_OK;
}

extern "C" void odwf_batch_destroy(odwf_batch B) {
  if (!B) return;
  (void)hipSetDevice(B->S->lat->device);
  (void)hipDeviceSynchronize();
  if (B->hscal) (void)hipHostFree(B->hscal);
  delete B;
}
