// Operator sequences and solvers built on the fused kernels.
#pragma once
#include "runtime.h"

namespace odwf {

// D = omega (A + W)(1 + L) on full fields given as (even, odd) halves;
// te/to are scratch halves.
hipError_t apply_D(const OpCtx& c, const HV& ie, const HV& io, const HV& te, const HV& to,
                   const HV& oe, const HV& oo);
// D^dag = (1 + L)^dag (A^dag + W^dag) omega
hipError_t apply_Ddag(const OpCtx& c, const HV& ie, const HV& io, const HV& te, const HV& to,
                      const HV& oe, const HV& oo);
// S_e in (to: odd scratch)
hipError_t apply_schur(const OpCtx& c, const HV& in, const HV& to, const HV& out);
// S_e^dag in
hipError_t apply_schur_dag(const OpCtx& c, const HV& in, const HV& te, const HV& to, const HV& out);

// Fused CG pieces of the normal operator N = S_e^dag S_e applied to p:
//   K1: t = A^{-1} W_oe p
//   K2: v = A^{-dag} (p - A^{-1} W_eo t), partial |S_e p|^2 (if partial_u)
//   K3: t = A^{-dag} W^dag_oe v
//   K4: out = A^dag v - W^dag_eo t
// With k4 options the last step can instead update r (r -= alpha N p, |r|^2) or write a
// residual f - N p.
hipError_t apply_normal(const OpCtx& c, const HV& p, const HV& t, const HV& v, const HV& out,
                        double* partial_u, const HopOpt* k4 = nullptr, const CGScal* gate = nullptr,
                        int gate_mode = GATE_NONE);

// how a solve chunk receives its source and returns its solution
struct SolveIO {
  bool bcast_b = false;      // b holds one right-hand side, the source of every one of the chunk
  void* y_packed = nullptr;  // EO_NORMAL: caller's packed FP64 even half (nrhs right-hand sides),
                             // used as the CG iterate and left holding the solution; x unused
};

odwf_status solve_chunk(odwf_solver S, int mode, const double* mq, const double* tol, int r0,
                        int nrhs, int inner, int maxiter, const void* b, void* x, int use_x0,
                        odwf_stats* stats, hipStream_t st, const SolveIO& io = SolveIO());

size_t solve_workspace_bytes(long h, int Ns, int nrhs, int inner);

// device buffers of a solve chunk of nrhs right-hand sides (named workspace
// entries, allocated on first use and kept)
struct SolveBufs {
  HV e0, e1, e2, o0;  // FP64: f, y, even scratch, odd scratch
  HV r, p, x, t, v;   // inner precision (FP64: r, p only)
  double* partial = nullptr;
  CGScal* scal = nullptr;
  double* res = nullptr;
};
bool solve_buffers(Workspace& W, long h, int nrhs, int Ns, int inner, SolveBufs& B, bool own_y = true);

}  // namespace odwf
