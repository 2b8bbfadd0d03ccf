// Operator sequences and conjugate-gradient solvers (paper §2: the solves
// behind the fermion forces are conjugate gradient on the normal operator).
//
// All solvers iterate textbook CG on N = S_e^dag S_e with device-resident
// scalars (one CGScal record per right-hand side): alpha and beta are formed
// on the device from deterministic FP64 reductions, so the host only polls
// convergence flags a couple of iterations behind the GPU.
//   FP64:        plain CG; the solution and residual are FP64.
//   FP32:        CG in FP32 storage/arithmetic with FP64 reliable updates:
//                when |r| drops below delta * max|r| since the last update,
//                or when the iterated residual meets tol, the FP32 increment is
//                added to the FP64 solution and the true residual f - N y is
//                recomputed with the FP64 operator.
//   FP16S/BF16S: FP64 defect correction: r = f - N y in FP64, an inner CG in
//                half/bfloat16 storage (per-site scales, FP32 arithmetic) solves
//                N e = r to a loose tolerance, y += e, repeat.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace odwf {

hipError_t apply_D(const OpCtx& c, const HV& ie, const HV& io, const HV& te, const HV& to,
                   const HV& oe, const HV& oo) {
  // y = (1 + L) psi; out = omega (A y_site + W y)
  HIPRET(m5(c, ie, te, prog_1pl()));
  HIPRET(m5(c, io, to, prog_1pl()));
  HopOpt o;
  o.px = prog_a();
  o.po = prog_omega();
  o.x = &te;
  HIPRET(hop(c, 0, 0, to, &oe, o));
  o.x = &to;
  HIPRET(hop(c, 1, 0, te, &oo, o));
  return hipSuccess;
}

hipError_t apply_Ddag(const OpCtx& c, const HV& ie, const HV& io, const HV& te, const HV& to,
                      const HV& oe, const HV& oo) {
  // y = omega psi; out = (1 + L)^dag (A^dag y_site + W^dag y)
  HIPRET(m5(c, ie, te, prog_omega()));
  HIPRET(m5(c, io, to, prog_omega()));
  HopOpt o;
  o.px = prog_a_t();
  o.po = prog_1pl_t();
  o.x = &te;
  HIPRET(hop(c, 0, 1, to, &oe, o));
  o.x = &to;
  HIPRET(hop(c, 1, 1, te, &oo, o));
  return hipSuccess;
}

hipError_t apply_schur(const OpCtx& c, const HV& in, const HV& to, const HV& out) {
  HopOpt k1;
  k1.ph = prog_ainv();
  HIPRET(hop(c, 1, 0, in, &to, k1));
  HopOpt k2;
  k2.ph = prog_ainv();
  k2.x = &in;
  k2.ch = -1.0;
  k2.cx = 1.0;
  return hop(c, 0, 0, to, &out, k2);
}

hipError_t apply_schur_dag(const OpCtx& c, const HV& in, const HV& te, const HV& to, const HV& out) {
  // S_e^dag = 1 - W^dag_eo A^{-dag} W^dag_oe A^{-dag}
  HIPRET(m5(c, in, te, prog_ainv_t()));
  HopOpt k3;
  k3.ph = prog_ainv_t();
  HIPRET(hop(c, 1, 1, te, &to, k3));
  HopOpt k4;
  k4.x = &in;
  k4.ch = -1.0;
  k4.cx = 1.0;
  return hop(c, 0, 1, to, &out, k4);
}

hipError_t apply_normal(const OpCtx& c, const HV& p, const HV& t, const HV& v, const HV& out,
                        double* partial_u, const HopOpt* k4opt, const CGScal* gate, int gate_mode) {
  HopOpt k1;
  k1.ph = prog_ainv();
  k1.gate = gate;
  k1.gate_mode = gate_mode;
  HIPRET(hop(c, 1, 0, p, &t, k1));
  HopOpt k2;
  k2.ph = prog_ainv();
  k2.x = &p;
  k2.ch = -1.0;
  k2.cx = 1.0;
  k2.po = prog_ainv_t();
  k2.partial = partial_u;
  k2.gate = gate;
  k2.gate_mode = gate_mode;
  HIPRET(hop(c, 0, 0, t, &v, k2));
  if (partial_u && k4opt && k4opt->scal && k4opt->cg_r)
    HIPRET(launch_fin(FIN_ALPHA, partial_u, hop_nblocks((int)c.h(), c.nrhs, c.Ns()), c.nrhs,
                      const_cast<CGScal*>(k4opt->scal), nullptr, c.st));
  HopOpt k3;
  k3.ph = prog_ainv_t();
  k3.gate = gate;
  k3.gate_mode = gate_mode;
  HIPRET(hop(c, 1, 1, v, &t, k3));
  HopOpt k4 = k4opt ? *k4opt : HopOpt();
  k4.x = &v;
  k4.px = prog_a_t();
  k4.ch = -1.0;
  k4.cx = 1.0;
  k4.gate = gate;
  k4.gate_mode = gate_mode;
  const HV* o = (k4opt && k4opt->cg_r) ? nullptr : &out;
  return hop(c, 0, 1, t, o, k4);
}

// ---------------------------------------------------------------------------
// host polling of the device scalars, a few iterations behind the GPU
// ---------------------------------------------------------------------------
struct Poller {
  CGScal* host = nullptr;  // pinned, 4 slots
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  long k = 0;
  hipError_t init() {
    HIPRET(hipHostMalloc((void**)&host, 4 * MAXRHS * sizeof(CGScal), hipHostMallocDefault));
    for (int i = 0; i < 4; i++) HIPRET(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    return hipSuccess;
  }
  ~Poller() {
    for (int i = 0; i < 4; i++)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (host) (void)hipHostFree(host);
  }
  hipError_t push(const CGScal* d, int nrhs, hipStream_t st) {
    const int slot = (int)(k % 4);
    // the slot's previous copy must have landed before it is overwritten
    if (k >= 4) HIPRET(hipEventSynchronize(ev[slot]));
    HIPRET(hipMemcpyAsync(host + slot * MAXRHS, d, nrhs * sizeof(CGScal), hipMemcpyDeviceToHost, st));
    HIPRET(hipEventRecord(ev[slot], st));
    k++;
    return hipSuccess;
  }
  // scalars as of `lag` pushes ago (nullptr if none yet)
  const CGScal* view(int lag) {
    if (k <= lag) return nullptr;
    const int slot = (int)((k - 1 - lag) % 4);
    if (hipEventSynchronize(ev[slot]) != hipSuccess) return nullptr;
    return host + slot * MAXRHS;
  }
};

static hipError_t read_scal(const CGScal* d, CGScal* h, int nrhs, hipStream_t st) {
  HIPRET(hipMemcpyAsync(h, d, nrhs * sizeof(CGScal), hipMemcpyDeviceToHost, st));
  return hipStreamSynchronize(st);
}

size_t solve_workspace_bytes(long h, int Ns, int nrhs, int inner) {
  size_t b = 4 * half_bytes(h, nrhs, Ns, PREC64);  // f, y, two FP64 temporaries
  if (inner == PREC64) {
    b += 2 * half_bytes(h, nrhs, Ns, PREC64);  // r, p
  } else {
    b += 5 * (half_bytes(h, nrhs, Ns, inner) + scale_bytes(h, nrhs, Ns, inner));
  }
  const int nb = std::max(hop_nblocks((int)h, nrhs, Ns), vec_nblocks(h, nrhs, Ns));
  b += partial_bytes(nb, nrhs) + 64 * 1024;
  return b;
}

bool solve_buffers(Workspace& W, long h, int nrhs, int Ns, int inner, SolveBufs& B, bool own_y) {
  B.e0 = W.half("s.e0", h, nrhs, Ns, PREC64);  // f
  if (own_y) B.e1 = W.half("s.e1", h, nrhs, Ns, PREC64);  // y (else the caller's packed field)
  B.e2 = W.half("s.e2", h, nrhs, Ns, PREC64);  // FP64 even scratch / residual
  B.o0 = W.half("s.o0", h, nrhs, Ns, PREC64);  // FP64 odd scratch
  const int nbmax = std::max(hop_nblocks((int)h, nrhs, Ns), vec_nblocks(h, nrhs, Ns));
  B.partial = (double*)W.get("s.partial", partial_bytes(nbmax, nrhs));
  B.scal = (CGScal*)W.get("s.scal", 2 * MAXRHS * sizeof(CGScal));
  B.res = (double*)W.get("s.res", 4 * MAXRHS * sizeof(double));
  bool ok = B.e0.d && (B.e1.d || !own_y) && B.e2.d && B.o0.d && B.partial && B.scal && B.res;
  if (inner == PREC64) {
    B.r = W.half("s.r64", h, nrhs, Ns, PREC64);
    B.p = W.half("s.p64", h, nrhs, Ns, PREC64);
    return ok && B.r.d && B.p.d;
  }
  B.p = W.half("s.p", h, nrhs, Ns, inner);
  B.r = W.half("s.r", h, nrhs, Ns, inner);
  B.x = W.half("s.x", h, nrhs, Ns, inner);
  B.t = W.half("s.t", h, nrhs, Ns, inner);
  B.v = W.half("s.v", h, nrhs, Ns, inner);
  return ok && B.p.d && B.r.d && B.x.d && B.t.d && B.v.d;
}

// residual f - N y into `res` (which may be the v scratch) and its norm
// partials; then FIN_INIT on scal
static hipError_t true_residual(const OpCtx& c64, const HV& f, const HV& y, const HV& t, const HV& v,
                                double* partial, CGScal* scal, double* out) {
  HopOpt k4;
  k4.partial = partial;
  k4.cg_p = &f;
  HIPRET(apply_normal(c64, y, t, v, v, nullptr, &k4));
  return launch_fin(FIN_INIT, partial, hop_nblocks((int)c64.h(), c64.nrhs, c64.Ns()), c64.nrhs,
                    scal, out, c64.st);
}

odwf_status solve_chunk(odwf_solver S, int mode, const double* mq, const double* tol, int r0,
                        int nrhs, int inner, int maxiter, const void* b, void* x, int use_x0,
                        odwf_stats* stats, hipStream_t st, const SolveIO& io) {
  const auto t0 = std::chrono::steady_clock::now();
  Workspace& W = S->workspace(st);
  const Geom& g = S->lat->g;
  const long h = g.h;
  const int Ns = S->Ns;
  OpCtx c64;
  c64.S = S;
  c64.st = st;
  c64.prec = PREC64;
  c64.nrhs = nrhs;
  for (int r = 0; r < MAXRHS; r++) c64.kappa[r] = r < nrhs ? -mq[r] / (2.0 * S->m0) : 0.0;
  OpCtx cin = c64;
  cin.prec = inner;

#define CHK(expr)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      set_error(std::string("odwf_solve: HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return ODWF_EHIP;                                                                 \
    }                                                                                   \
  } while (0)

  SolveBufs B;
  if (!solve_buffers(W, h, nrhs, Ns, inner, B, io.y_packed == nullptr)) {
    set_error("odwf_solve: out of device memory for workspaces");
    return ODWF_ENOMEM;
  }
  if (io.y_packed) {  // the caller's packed even half is the CG iterate itself
    B.e1.d = io.y_packed;
    B.e1.sc = nullptr;
    B.e1.prec = PREC64;
  }
  HV e0 = B.e0, e1 = B.e1, e2 = B.e2, o0 = B.o0;
  double* partial = B.partial;
  CGScal* dscal = B.scal;
  CGScal* dscal_out = dscal + MAXRHS;
  double* dres = B.res;
  int nb_vec = 0;

  // ---- right-hand side f of the iterated system, initial guess y ----------
  if (mode == ODWF_SOLVE_FULL) {
    // b' = omega^{-1} b; phi_e = A^{-1}(b'_e - W_eo A^{-1} b'_o); f = S_e^dag phi_e
    CHK(launch_pack_spinor(PREC64, b, r0, e2.d, nullptr, 0, nrhs, Ns, g, st));
    CHK(launch_pack_spinor(PREC64, b, r0, o0.d, nullptr, 1, nrhs, Ns, g, st));
    CHK(m5(c64, e2, e2, prog_omega_inv()));
    CHK(m5(c64, o0, o0, prog_omega_inv()));
    CHK(m5(c64, o0, o0, prog_ainv()));
    HopOpt k;
    k.x = &e2;
    k.ch = -1.0;
    k.cx = 1.0;
    k.po = prog_ainv();
    CHK(hop(c64, 0, 0, o0, &e1, k));  // phi in e1
    CHK(apply_schur_dag(c64, e1, e2, o0, e0));
    if (use_x0) {
      CHK(launch_pack_spinor(PREC64, x, r0, e1.d, nullptr, 0, nrhs, Ns, g, st));
      CHK(m5(c64, e1, e1, prog_1pl()));
    } else {
      CHK(launch_vec_zero(PREC64, e1.d, nullptr, h, nrhs, Ns, st));
    }
  } else {
    if (io.bcast_b) {
      // one source for every right-hand side of the chunk (several masses)
      CHK(launch_pack_spinor(PREC64, b, 0, o0.d, nullptr, 0, 1, Ns, g, st));
      for (int q = 0; q < nrhs; q++)
        CHK(launch_vec_copy_rhs(PREC64, o0.d, nullptr, 1, 0, PREC64, e0.d, nullptr, nrhs, q, h, Ns, st));
    } else {
      CHK(launch_pack_spinor(PREC64, b, r0, e0.d, nullptr, 0, nrhs, Ns, g, st));
    }
    if (io.y_packed) {
      if (!use_x0) CHK(launch_vec_zero(PREC64, e1.d, nullptr, h, nrhs, Ns, st));
    } else if (use_x0) {
      CHK(launch_pack_spinor(PREC64, x, r0, e1.d, nullptr, 0, nrhs, Ns, g, st));
    } else {
      CHK(launch_vec_zero(PREC64, e1.d, nullptr, h, nrhs, Ns, st));
    }
  }

  // ---- device scalars --------------------------------------------------------
  CGScal hs[2 * MAXRHS];
  std::memset(hs, 0, sizeof(hs));
  for (int r = 0; r < nrhs; r++) {
    hs[r].tol2 = tol[r] * tol[r];
    hs[r].maxiter = maxiter;
    hs[r].active = 1;
    hs[r].delta2 = inner == PREC32 ? RELIABLE_DELTA2 : 0.0;
    hs[MAXRHS + r] = hs[r];
    hs[MAXRHS + r].delta2 = 0.0;
  }
  CHK(hipMemcpyAsync(dscal, hs, sizeof(hs), hipMemcpyHostToDevice, st));
  CHK(launch_vec_norm2(PREC64, e0.d, nullptr, partial, h, nrhs, Ns, &nb_vec, st));
  CHK(launch_fin(FIN_F2, partial, nb_vec, nrhs, dscal, nullptr, st));
  CHK(launch_fin(FIN_F2, partial, nb_vec, nrhs, dscal_out, nullptr, st));

  Poller poll;
  CHK(poll.init());
  CGScal cur[MAXRHS];
  int reliable = 0, outer = 0;
  std::vector<int> inner_iters(nrhs, 0), outer_q(nrhs, 0);
  // per right-hand side: seconds from the call's start until it was first seen finished
  std::vector<double> t_done(nrhs, -1.0);
  auto mark_done = [&]() {
    const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < nrhs; q++)
      if (t_done[q] < 0 && !cur[q].active) t_done[q] = now;
  };

  // initial true residual r = f - N y (or r = f from a zero guess)
  auto init_residual = [&](CGScal* sc) -> hipError_t {
    if (use_x0 || outer > 0 || reliable > 0) return true_residual(c64, e0, e1, o0, e2, partial, sc, dres);
    HIPRET(launch_vec_convert(PREC64, e0.d, nullptr, PREC64, e2.d, nullptr, 0, h, nrhs, Ns, st));
    HIPRET(launch_vec_norm2(PREC64, e2.d, nullptr, partial, h, nrhs, Ns, &nb_vec, st));
    return launch_fin(FIN_INIT, partial, nb_vec, nrhs, sc, dres, st);
  };

  const int nbh = hop_nblocks((int)h, nrhs, Ns);
  auto any = [&](const CGScal* s, int which) {
    for (int r = 0; r < nrhs; r++) {
      if (which == 0 && s[r].active) return true;
      if (which == 1 && s[r].update) return true;
    }
    return false;
  };

  if (inner == PREC64) {
    HV r = B.r, p = B.p;
    CHK(init_residual(dscal));
    CHK(launch_vec_convert(PREC64, e2.d, nullptr, PREC64, r.d, nullptr, 0, h, nrhs, Ns, st));
    CHK(launch_vec_convert(PREC64, r.d, nullptr, PREC64, p.d, nullptr, 0, h, nrhs, Ns, st));
    CHK(read_scal(dscal, cur, nrhs, st));
    while (any(cur, 0)) {
      for (;;) {
        HopOpt k4;
        k4.cg_r = &r;
        k4.scal = dscal;
        k4.partial = partial;
        CHK(apply_normal(c64, p, o0, e2, e2, partial, &k4));
        CHK(launch_fin(FIN_BETA, partial, nbh, nrhs, dscal, nullptr, st));
        CHK(launch_vec_cg_step(PREC64, r.d, nullptr, p.d, nullptr, e1.d, nullptr, dscal, h, nrhs, Ns, st));
        CHK(poll.push(dscal, nrhs, st));
        const CGScal* v = poll.view(2);
        if (v && !any(v, 0)) break;
      }
      // confirm with the true residual; continue where it has drifted
      CHK(true_residual(c64, e0, e1, o0, e2, partial, dscal, dres));
      CHK(launch_vec_convert(PREC64, e2.d, nullptr, PREC64, r.d, nullptr, 0, h, nrhs, Ns, st));
      CHK(read_scal(dscal, cur, nrhs, st));
      mark_done();
      reliable++;
    }
    for (int q = 0; q < nrhs; q++) inner_iters[q] = cur[q].iters;
  } else if (inner == PREC32) {
    HV p = B.p, rr = B.r, xs = B.x, t = B.t, v = B.v;
    CHK(init_residual(dscal));
    CHK(launch_vec_convert(PREC64, e2.d, nullptr, inner, rr.d, rr.sc, 0, h, nrhs, Ns, st));
    CHK(launch_vec_convert(inner, rr.d, rr.sc, inner, p.d, p.sc, 0, h, nrhs, Ns, st));
    CHK(launch_vec_zero(inner, xs.d, xs.sc, h, nrhs, Ns, st));
    CHK(read_scal(dscal, cur, nrhs, st));
    while (any(cur, 0)) {
      for (;;) {
        HopOpt k4;
        k4.cg_r = &rr;
        k4.scal = dscal;
        k4.partial = partial;
        CHK(apply_normal(cin, p, t, v, v, partial, &k4));
        CHK(launch_fin(FIN_BETA, partial, nbh, nrhs, dscal, nullptr, st));
        CHK(launch_vec_cg_step(inner, rr.d, rr.sc, p.d, p.sc, xs.d, xs.sc, dscal, h, nrhs, Ns, st));
        CHK(poll.push(dscal, nrhs, st));
        const CGScal* vw = poll.view(2);
        if (vw && (!any(vw, 0) || any(vw, 1))) break;
      }
      // reliable update: y += x_s, r = f - N y in FP64, restart the FP32 residual
      CHK(launch_vec_convert(inner, xs.d, xs.sc, PREC64, e1.d, nullptr, 1, h, nrhs, Ns, st));
      CHK(launch_vec_zero(inner, xs.d, xs.sc, h, nrhs, Ns, st));
      CHK(true_residual(c64, e0, e1, o0, e2, partial, dscal, dres));
      CHK(launch_vec_convert(PREC64, e2.d, nullptr, inner, rr.d, rr.sc, 0, h, nrhs, Ns, st));
      CHK(read_scal(dscal, cur, nrhs, st));
      mark_done();
      reliable++;
    }
    for (int q = 0; q < nrhs; q++) inner_iters[q] = cur[q].iters;
  } else {
    // defect correction around a half/bfloat16 inner CG
    HV p = B.p, rr = B.r, xs = B.x, t = B.t, v = B.v;
    const double tol_in = inner == PREC16 ? 5e-3 : 2e-2;
    CHK(init_residual(dscal_out));
    CHK(read_scal(dscal_out, cur, nrhs, st));
    while (any(cur, 0)) {
      for (int q = 0; q < nrhs; q++) outer_q[q] += cur[q].active ? 1 : 0;
      // inner system N e = r, started from e = 0
      CGScal hin[MAXRHS];
      for (int q = 0; q < nrhs; q++) {
        hin[q] = cur[q];
        hin[q].f2 = cur[q].rr;
        hin[q].tol2 = std::max(tol_in * tol_in, cur[q].tol2 * cur[q].f2 / std::max(cur[q].rr, 1e-300));
        hin[q].maxiter = std::max(1, maxiter - inner_iters[q]);
        hin[q].iters = 0;
        hin[q].converged = 0;
        hin[q].update = 0;
        hin[q].delta2 = 0.0;
        hin[q].rmax2 = cur[q].rr;
        hin[q].active = cur[q].active;
      }
      CHK(hipMemcpyAsync(dscal, hin, nrhs * sizeof(CGScal), hipMemcpyHostToDevice, st));
      CHK(launch_vec_convert(PREC64, e2.d, nullptr, inner, rr.d, rr.sc, 0, h, nrhs, Ns, st));
      CHK(launch_vec_convert(inner, rr.d, rr.sc, inner, p.d, p.sc, 0, h, nrhs, Ns, st));
      CHK(launch_vec_zero(inner, xs.d, xs.sc, h, nrhs, Ns, st));
      for (;;) {
        HopOpt k4;
        k4.cg_r = &rr;
        k4.scal = dscal;
        k4.partial = partial;
        CHK(apply_normal(cin, p, t, v, v, partial, &k4));
        CHK(launch_fin(FIN_BETA, partial, nbh, nrhs, dscal, nullptr, st));
        CHK(launch_vec_cg_step(inner, rr.d, rr.sc, p.d, p.sc, xs.d, xs.sc, dscal, h, nrhs, Ns, st));
        CHK(poll.push(dscal, nrhs, st));
        const CGScal* vw = poll.view(2);
        if (vw && !any(vw, 0)) break;
      }
      CGScal fin[MAXRHS];
      CHK(read_scal(dscal, fin, nrhs, st));
      for (int q = 0; q < nrhs; q++) inner_iters[q] += fin[q].iters;
      CHK(launch_vec_convert(inner, xs.d, xs.sc, PREC64, e1.d, nullptr, 1, h, nrhs, Ns, st));
      outer++;
      // outer residual; carry the iteration count so maxiter bounds the total
      for (int q = 0; q < nrhs; q++) cur[q].iters = inner_iters[q];
      CHK(hipMemcpyAsync(dscal_out, cur, nrhs * sizeof(CGScal), hipMemcpyHostToDevice, st));
      CHK(true_residual(c64, e0, e1, o0, e2, partial, dscal_out, dres));
      CHK(read_scal(dscal_out, cur, nrhs, st));
      mark_done();
      for (int q = 0; q < nrhs; q++)
        if (fin[q].nan) cur[q].nan = 1, cur[q].active = 0;
    }
  }

  // ---- output ----------------------------------------------------------------
  double full_res[MAXRHS];
  for (int q = 0; q < nrhs; q++) full_res[q] = -1.0;
  if (mode == ODWF_SOLVE_FULL) {
    // y_o = A^{-1}(b'_o - W_oe y_e)
    CHK(launch_pack_spinor(PREC64, b, r0, o0.d, nullptr, 1, nrhs, Ns, g, st));
    CHK(m5(c64, o0, o0, prog_omega_inv()));
    HopOpt k;
    k.x = &o0;
    k.ch = -1.0;
    k.cx = 1.0;
    k.po = prog_ainv();
    CHK(hop(c64, 1, 0, e1, &o0, k));
    // |b - D x| with D x = omega (A + W) y, parity by parity (e0 reused as scratch)
    double nr[MAXRHS], nb2[MAXRHS];
    for (int q = 0; q < nrhs; q++) nr[q] = nb2[q] = 0.0;
    for (int par = 0; par < 2; par++) {
      HopOpt kd;
      kd.px = prog_a();
      kd.po = prog_omega();
      kd.x = par == 0 ? &e1 : &o0;
      CHK(hop(c64, par, 0, par == 0 ? o0 : e1, &e0, kd));
      CHK(launch_pack_spinor(PREC64, b, r0, e2.d, nullptr, par, nrhs, Ns, g, st));
      CHK(launch_vec_norm2(PREC64, e2.d, nullptr, partial, h, nrhs, Ns, &nb_vec, st));
      CHK(launch_fin(FIN_SUM, partial, nb_vec, nrhs, nullptr, dres + 2 * MAXRHS, st));
      CHK(m5(c64, e0, e0, prog_none(), -1.0, &e2, 1.0));
      CHK(launch_vec_norm2(PREC64, e0.d, nullptr, partial, h, nrhs, Ns, &nb_vec, st));
      CHK(launch_fin(FIN_SUM, partial, nb_vec, nrhs, nullptr, dres + MAXRHS, st));
      double hr[4 * MAXRHS];
      CHK(hipMemcpyAsync(hr, dres, sizeof(hr), hipMemcpyDeviceToHost, st));
      CHK(hipStreamSynchronize(st));
      for (int q = 0; q < nrhs; q++) {
        nr[q] += hr[MAXRHS + q];
        nb2[q] += hr[2 * MAXRHS + q];
      }
    }
    for (int q = 0; q < nrhs; q++) full_res[q] = nb2[q] > 0 ? std::sqrt(nr[q] / nb2[q]) : 0.0;
    // x = (1 + L)^{-1} y
    CHK(m5(c64, e1, e1, prog_1pl_inv()));
    CHK(m5(c64, o0, o0, prog_1pl_inv()));
    CHK(launch_unpack_spinor(PREC64, e1.d, nullptr, x, r0, 0, nrhs, Ns, g, st));
    CHK(launch_unpack_spinor(PREC64, o0.d, nullptr, x, r0, 1, nrhs, Ns, g, st));
  } else if (!io.y_packed) {
    CHK(launch_unpack_spinor(PREC64, e1.d, nullptr, x, r0, 0, nrhs, Ns, g, st));
    CHK(launch_zero_canon_parity(x, r0, 1, nrhs, Ns, g, st));
  }
  CHK(hipStreamSynchronize(st));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

  odwf_status worst = ODWF_OK;
  for (int q = 0; q < nrhs; q++) {
    const double rel = cur[q].f2 > 0 ? std::sqrt(cur[q].rr / cur[q].f2) : 0.0;
    int stq = ODWF_OK;
    if (cur[q].nan || !std::isfinite(rel)) stq = ODWF_ENAN;
    else if (!cur[q].converged) stq = ODWF_ENOCONV;
    if (stq == ODWF_ENAN) worst = ODWF_ENAN;
    else if (stq == ODWF_ENOCONV && worst == ODWF_OK) worst = ODWF_ENOCONV;
    if (stats) {
      stats[q].iters = inner_iters[q];
      // FP32: the FP64 true-residual updates of this right-hand side's own iterate
      stats[q].reliable_updates = inner == PREC32 ? cur[q].nupd : 0;
      stats[q].outer_steps = outer_q[q];
      stats[q].status = stq;
      stats[q].true_rel_resid = rel;
      stats[q].full_rel_resid = full_res[q];
      stats[q].seconds = t_done[q] >= 0 && t_done[q] < secs ? t_done[q] : secs;
    }
  }
  if (worst == ODWF_ENAN) set_error("odwf_solve: NaN/Inf in a residual norm");
  else if (worst == ODWF_ENOCONV) set_error("odwf_solve: maxiter reached before tol");
  return worst;
#undef CHK
}

}  // namespace odwf
