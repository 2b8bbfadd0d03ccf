// Host runtime of libodwf: lattice and solver objects, workspaces, operator
// sequences built from the kernels, and the solvers.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/odwf.h"
#include "kernels.h"
#include "odwf_types.h"

#define HIPRET(expr)                 \
  do {                               \
    hipError_t e_ = (expr);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

namespace odwf {

void set_error(const std::string& msg);

// a device buffer that the library owns
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// one half field (even or odd sites) in a storage precision
struct HV {
  void* d = nullptr;
  float* sc = nullptr;  // per-5D-site scales (FP16S / BF16S)
  int prec = PREC64;
};

size_t bytes_per_complex(int prec);
size_t half_bytes(long h, int nrhs, int Ns, int prec);   // data
size_t scale_bytes(long h, int nrhs, int Ns, int prec);  // scales (0 if unscaled)

// per-stream cache of named device buffers
struct Workspace {
  std::map<std::string, DevBuf> bufs;
  ~Workspace();
  void* get(const std::string& name, size_t bytes);
  HV half(const std::string& name, long h, int nrhs, int Ns, int prec);
  size_t total() const;
};

}  // namespace odwf

struct odwf_lattice_s {
  int dims[4];
  int bc_t;
  int device;
  odwf::Geom g;
  void* U64[2] = {nullptr, nullptr};  // per output parity, [h][8][18] double
  void* U32[2] = {nullptr, nullptr};  // per output parity, [h][8][12] float
  bool loaded = false;
};

struct odwf_solver_s {
  odwf_lattice lat;
  int Ns;
  double m0;
  std::vector<double> omega;
  void* coef64 = nullptr;  // [2][NCOEF][Ns] double
  void* coef32 = nullptr;  // [2][NCOEF][Ns] float
  std::mutex mtx;
  std::map<hipStream_t, odwf::Workspace*> ws;
  odwf::Workspace& workspace(hipStream_t st);
};

namespace odwf {

// programs of the fifth-dimension operators
M5Prog prog_none();
M5Prog prog_ainv();      // A^{-1}
M5Prog prog_ainv_t();    // A^{-dag} (A is real per chirality)
M5Prog prog_a();         // A
M5Prog prog_a_t();       // A^dag
M5Prog prog_omega();
M5Prog prog_omega_inv();
M5Prog prog_1pl();       // 1 + L
M5Prog prog_1pl_inv();   // (1 + L)^{-1}
M5Prog prog_1pl_t();     // (1 + L)^dag

// per-call operator context (one chunk of <= MAXRHS right-hand sides)
struct OpCtx {
  odwf_solver S;
  hipStream_t st;
  int prec;  // storage precision of the half fields passed to the helpers
  int nrhs;
  double kappa[MAXRHS];
  bool noprof = false;  // never record profiling events (the allocation-free path)
  const void* coef() const { return prec == PREC64 ? S->coef64 : S->coef32; }
  const void* links(int par) const { return prec == PREC64 ? S->lat->U64[par] : S->lat->U32[par]; }
  long h() const { return S->lat->g.h; }
  int Ns() const { return S->Ns; }
};

struct HopOpt {
  const HV* x = nullptr;
  M5Prog ph, px, po;
  double ch = 1.0, cx = 1.0;
  // CG fusion
  double* partial = nullptr;
  HV* cg_r = nullptr;
  const HV* cg_p = nullptr;  // f of the residual f - N p (mode 3)
  const CGScal* scal = nullptr;
  // gating (GateMode): only right-hand sides selected by gate do any work
  const CGScal* gate = nullptr;
  int gate_mode = GATE_NONE;
  HopOpt() : ph(prog_none()), px(prog_none()), po(prog_none()) {}
};

hipError_t hop(const OpCtx& c, int out_par, int dag, const HV& in, const HV* out, const HopOpt& o);
hipError_t m5(const OpCtx& c, const HV& in, const HV& out, const M5Prog& p, double c0 = 1.0,
              const HV* other = nullptr, double c1 = 0.0);

// profiler hooks
void prof_begin(hipStream_t st, int key);
void prof_end(hipStream_t st, double bytes);
bool prof_on();

}  // namespace odwf
