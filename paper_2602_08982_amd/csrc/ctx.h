// Context of libtdslda and the per-shape kernel-set interface (shared by
// the C-ABI translation unit and the engine instantiation units).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tdslda.h"
#include "kernels3d.h"

namespace tdslda {

// ----------------------------------------------------------------------------
// kernel classes for the profiling counters
enum KClass {
  KC_DENS = 0, KC_REDUCE_POT, KC_LAP1, KC_FINALIZE, KC_LAP2_CORR, KC_LAP2_FULL, KC_LAP2_F,
  KC_LAP2_H, KC_LAP2_TAYLOR, KC_PRED, KC_NORM, KC_GRAD, KC_ENERGY, KC_SETUP, KC_Q1D_FUSED,
  KC_DENS_KIN, KC_FRICTION, KC_COUNT
};
inline const char* const kKernelNames[KC_COUNT] = {
    "dens", "reduce_pot", "lap1", "finalize", "lap2_corr", "lap2_full", "lap2_f", "lap2_h",
    "lap2_taylor", "pred", "norm", "grad", "energy", "setup", "q1d_fused", "dens_kin", "friction"};

struct Fail {
  tdslda_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw Fail{TDSLDA_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};      \
  } while (0)

inline void require(bool ok, tdslda_status st, const std::string& msg) {
  if (!ok) throw Fail{st, msg};
}

struct L2Desc {
  int mode = L2_H;
  const void* X = nullptr;
  void* Xout = nullptr;
  const void* T = nullptr;
  const double* scale = nullptr;
  const double* hshift = nullptr;
  void* out = nullptr;
  void* acc = nullptr;
  const void* hist[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  void* cout = nullptr;
  double* nrm_part = nullptr;
  double tay_re = 0, tay_im = 0;
  int init_acc = 0;
};

struct PwDesc {
  int mode = PW_NORM;
  void* X = nullptr;
  const double* scale = nullptr;
  const void* hist[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  void* cout = nullptr;
  double* nrm_part = nullptr;
  void* out64 = nullptr;
};

using Ctx = ::tdslda_ctx;

// Per-shape / per-precision kernel set.
struct Engine {
  virtual ~Engine() = default;
  virtual int ngx() const = 0;    // norm-partial slots per state (slab groups)
  virtual int ncb() const = 0;    // lap1 column blocks per state
  virtual int group() const = 0;  // states per density group
  virtual void dens(Ctx& c, const void* X, const double* scale, int64_t nst) = 0;
  // densities only, for a buffer whose (y,z) kinetic <H> partials were left
  // in the h slots by the kernel that wrote it (see producer_kinetic)
  virtual void dens_sum(Ctx& c, const void* X, const double* scale, int64_t nst) { dens(c, X, scale, nst); }
  // true when CORR / FULL write the kinetic partials of their output
  virtual bool producer_kinetic() const { return false; }
  // h slots that hold partials of the unscaled state
  virtual int raw_h_slots() const { return 0; }
  // true when lap2 in the F / CORR / FULL modes takes <H>_n of its input
  // itself (the whole state in one workgroup): those evaluations then need
  // the fields only, no lap1 and no shift
  virtual bool self_shift() const { return false; }
  // choose launch shapes by timing them on the loaded states; returns the
  // number of kernel classes tuned (0: this kernel set has no choices)
  virtual int autotune(Ctx& c, int32_t* out, double* ms_out) { (void)c; (void)out; (void)ms_out; return 0; }
  virtual void reduce_pot(Ctx& c, bool update) = 0;
  virtual void lap1(Ctx& c, const void* X, const double* scale, bool hpart, int64_t nst) = 0;
  virtual void lap2(Ctx& c, const L2Desc& d, int64_t nst) = 0;
  virtual void pointwise(Ctx& c, const PwDesc& d, int64_t nst) = 0;
  virtual void grad(Ctx& c, const void* X, const double* scale, int64_t n0, int64_t nchunk) = 0;
  // quantum friction: add the dissipative terms to the fields just built
  // from the states X (the quasi-1D and full-3D kernel sets have it)
  virtual void friction(Ctx& c, const void* X, const double* scale, int64_t nst) {
    (void)c, (void)X, (void)scale, (void)nst;
    throw Fail{TDSLDA_EINVAL, "quantum friction is built for the quasi-1D kernel set"};
  }
  virtual size_t elem_size() const = 0;
};

}  // namespace tdslda

using namespace tdslda;

struct tdslda_ctx {
  tdslda_lattice lat{};
  tdslda_functional fun{};
  tdslda_run run{};
  int q1d = 0, q2d = 0;
  int64_t M = 0, cap = 0, nst = 0;
  double dV = 1, dVe = 1, vol = 1, ainv = 1;
  hipStream_t stream = nullptr;
  std::unique_ptr<Engine> eng;
  size_t esz = 16;
  int depth = 4, np = 4, nq = 5;
  double bco[5] = {0}, aco[5] = {0};

  // device memory
  std::vector<void*> allocs;
  void* sb[6] = {nullptr};
  double* sscale[6] = {nullptr};
  void* T = nullptr;
  double *wu = nullptr, *wv = nullptr, *E = nullptr, *kperp2 = nullptr;
  double* mult = nullptr;  // per-state multiplicity (weights are mult f(+-E))
  double *nrm_part = nullptr, *h_part = nullptr, *hshift = nullptr;
  int nrm_stride = 1, h_stride = 1;
  double* dens_part = nullptr;
  int nsg_max = 1, nsg_used = 1, njg_used = 1;
  double *rho = nullptr, *nu = nullptr, *tau = nullptr, *jc = nullptr;
  double *U = nullptr, *delta = nullptr, *vext = nullptr, *lam = nullptr, *theta = nullptr;
  double* dext = nullptr;  // external pairing potential [M][2] (zero unless set)
  bool dext_on = false;
  void *hA = nullptr, *hD = nullptr;
  // general functional (A != 1, Eq. h_sigma; quasi-1D kernel set): inverse
  // effective mass alpha, its D2, and the current potential A_z, [M] in the
  // context precision; gen = the general operator is in use
  void *hAl = nullptr, *hLa = nullptr, *hAz = nullptr;
  void *hAx = nullptr, *hAy = nullptr;  // 3D: the x and y components of A
  double* jpart = nullptr;              // 3D: current group partials [group][3][M]
  bool gen = false;
  // spin-imbalanced ASLDA (quasi-1D kernel set): both branches evolved,
  // spin-resolved densities and fields ([spin][M] for rho, tau, j, U and
  // the fields of H)
  bool aslda = false;
  double* circ = nullptr;  // 3D ASLDA: the D2 circulants of the x, y, z axes (for Laplacians of alpha_s)
  double* gscratch = nullptr;  // [gchunk][4][M] doubles (tau_s, j_s); also FP64 staging
  int64_t gchunk = 1;
  double* eout = nullptr;
  int* dflag = nullptr;
  int32_t* kidx_dev = nullptr;
  int64_t kidx_cap = 0;
  // quantum friction (quasi-1D): parameters, group partials [group][3][M]
  // (j_z, Re B', Im B'), summed fields j[M], B'[M][2]
  bool fric = false;
  double f_alpha = 0, f_beta = 0, f_gamma = 0, f_rho0 = 1, f_Nreq = 0;
  double *fric_part = nullptr, *fric_j = nullptr, *fric_bp = nullptr;
  double *fric_div = nullptr, *fric_N = nullptr;  // 3D: div j [M], N

  // integrator state
  bool kin_ready[6] = {false, false, false, false, false, false};  // h slots hold this buffer's partials
  int phi = 0;
  int hist[5] = {1, 2, 3, 4, 5};
  bool loaded = false, started = false, frozen = false, fields_valid = false;
  int64_t steps = 0;
  double time = 0;
  bool have_ref = false;
  double N0 = 0, E0 = 0;

  // profiling
  bool prof = false;
  struct Ev {
    int k;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
  std::vector<hipEvent_t> pool;
  int64_t klaunch[KC_COUNT] = {0};
  double kms[KC_COUNT] = {0};

  std::string err;

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{TDSLDA_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    allocs.push_back(p);
    return p;
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  // bracket a launch with events when profiling
  template <class F>
  void launch(int k, F&& f) {
    if (prof) {
      hipEvent_t a = ev(), b = ev();
      HIPCHK(hipEventRecord(a, stream));
      f();
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(b, stream));
      events.push_back({k, a, b});
    } else {
      f();
      HIPCHK(hipGetLastError());
    }
#ifdef TDSLDA_DEBUG_SYNC
    HIPCHK(hipStreamSynchronize(stream));
#endif
  }
  void harvest() {
    for (auto& e : events) {
      HIPCHK(hipEventSynchronize(e.b));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
      klaunch[e.k] += 1;
      kms[e.k] += ms;
      pool.push_back(e.a);
      pool.push_back(e.b);
    }
    events.clear();
  }
  StateScalars scalars(double* scale) {
    StateScalars s;
    s.nrm_part = nrm_part;
    s.nrm_stride = nrm_stride;
    s.h_part = h_part;
    s.h_stride = h_stride;
    s.h_lap1_off = eng->ngx();
    s.scale = scale;
    s.hshift = hshift;
    return s;
  }
  // abm_graph: the private capture stream (when the context uses the null
  // stream) and the last executable graph, kept until the next abm_graph
  // call or the context's destruction instead of being released right after
  // the launch
  hipStream_t graph_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  void release_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~tdslda_ctx() {
    if (graph_exec || graph_stream) (void)hipDeviceSynchronize();
    release_graph();
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    for (auto& e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace tdslda {
inline unsigned cdiv(int64_t a, int64_t b) { return unsigned((a + b - 1) / b); }

// factories of the instantiation units (nullptr when the shape is not theirs)
std::unique_ptr<Engine> make3d_f64_small(int nx, int ny, int nz);
std::unique_ptr<Engine> make3d_f64_large(int nx, int ny, int nz);
std::unique_ptr<Engine> make3d_f32_small(int nx, int ny, int nz);
std::unique_ptr<Engine> make3d_f32_large(int nx, int ny, int nz);
std::unique_ptr<Engine> make_q1d_f64(int nz);
std::unique_ptr<Engine> make_q1d_f32(int nz);
std::unique_ptr<Engine> make_q2d_f64(int nx, int ny);
std::unique_ptr<Engine> make_q2d_f32(int nx, int ny);
// quasi-1D static states (q1dstatic.hip): counts per problem and, when X is
// given, the kept eigenvectors written at X (slots 0 .. total-1) with E and
// k_perp^2 per slot; returns the total number kept
int64_t q1d_static(hipStream_t st, int N, double dz, int nprob, const double* kperp2, const double* hfield,
                   const double* delta, double ecut, int32_t* counts, void* X, size_t esz, double* E_dev,
                   double* kp_dev, int64_t cap, const double* hfield_b = nullptr, bool both = false);
struct StaticSolver;
}  // namespace tdslda
