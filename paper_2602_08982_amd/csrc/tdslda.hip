// libtdslda: host side of the C ABI declared in include/tdslda.h.
//
// A context owns (history depth + 1) state buffers, the intermediate buffer
// T (x-derivative of every state) and the FP64 fields.  The integrator
// keeps buffer roles by index: phi (current state, raw with a per-buffer
// normalisation scale) and hist[0..D-1] (f_{k-1}, ..., f_{k-D}).  One ABM
// step is two right-hand-side evaluations, each
//     dens -> reduce_pot -> lap1 -> finalize(<H>) -> lap2(mode),
// (dens -> reduce_pot -> lap2 where a state fits one workgroup and lap2
// takes <H>_n itself), where lap2 fuses H.psi, the shift and the integrator
// arithmetic
// (Alg. AB4AM5: the corrector after the first evaluation, the next step's
// predictor and partial corrector after the second).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels_host.h"
#include "kernels3d_gen.h"

namespace tdslda {
std::vector<double> spectral_d2_circulant(int N, double dz);  // q1dstatic.hip
}

namespace {

std::unique_ptr<Engine> make_engine(const tdslda_lattice& lat, int prec) {
  std::unique_ptr<Engine> e;
  if (lat.mode == TDSLDA_MODE_3D) {
    if (prec == TDSLDA_FP64) {
      e = make3d_f64_small(lat.nx, lat.ny, lat.nz);
      if (!e) e = make3d_f64_large(lat.nx, lat.ny, lat.nz);
    } else {
      e = make3d_f32_small(lat.nx, lat.ny, lat.nz);
      if (!e) e = make3d_f32_large(lat.nx, lat.ny, lat.nz);
    }
  } else if (lat.mode == TDSLDA_MODE_Q2D) {
    e = prec == TDSLDA_FP64 ? make_q2d_f64(lat.nx, lat.ny) : make_q2d_f32(lat.nx, lat.ny);
  } else {
    e = prec == TDSLDA_FP64 ? make_q1d_f64(lat.nz) : make_q1d_f32(lat.nz);
  }
  return e;
}

// integrator constants (Eqs. AB3-AB5, AM4-AM5)
void set_scheme(Ctx& c) {
  static const double ab3[] = {23.0 / 12, -16.0 / 12, 5.0 / 12};
  static const double ab4[] = {55.0 / 24, -59.0 / 24, 37.0 / 24, -9.0 / 24};
  static const double ab5[] = {1901.0 / 720, -2774.0 / 720, 2616.0 / 720, -1274.0 / 720, 251.0 / 720};
  static const double am4[] = {9.0 / 24, 19.0 / 24, -5.0 / 24, 1.0 / 24};
  static const double am5[] = {251.0 / 720, 646.0 / 720, -264.0 / 720, 106.0 / 720, -19.0 / 720};
  const double* b;
  const double* a;
  switch (c.run.integrator) {
    case TDSLDA_AB3AM4: c.np = 3; c.nq = 4; b = ab3; a = am4; break;
    case TDSLDA_AB5AM5: c.np = 5; c.nq = 5; b = ab5; a = am5; break;
    case TDSLDA_AB4AM5: c.np = 4; c.nq = 5; b = ab4; a = am5; break;
    default: throw Fail{TDSLDA_EINVAL, "unknown integrator"};
  }
  c.depth = std::max(c.np, c.nq - 1);
  for (int i = 0; i < 5; ++i) {
    c.bco[i] = i < c.np ? c.run.dt * b[i] : 0.0;
    c.aco[i] = i < c.nq ? c.run.dt * a[i] : 0.0;
  }
}

int64_t memory_bytes(const tdslda_lattice& lat, const tdslda_run& run, int64_t n, Engine* eng,
                     int depth, int64_t gchunk) {
  const int64_t M = lat.mode == TDSLDA_MODE_3D    ? int64_t(lat.nx) * lat.ny * lat.nz
                    : lat.mode == TDSLDA_MODE_Q2D ? int64_t(lat.nx) * lat.ny
                                                  : lat.nz;
  const int64_t es = int64_t(eng->elem_size());
  const int64_t S = 2 * M * es;
  int64_t b = (depth + (lat.mode == TDSLDA_MODE_Q2D ? 1 : 2)) * n * S;  // state buffers + T
  b += n * 8 * (5 + (depth + 1) + 1);                            // per-state arrays
  b += n * 8 * (eng->ngx() + eng->ngx() + eng->ncb());           // partial slots
  b += int64_t(cdiv(n, eng->group())) * 3 * M * 8 * (lat.mode == TDSLDA_MODE_3D ? 2 : 1);  // density (+ current) partials
  b += M * 8 * 16 + M * (es / 2 + es);                          // fields
  b += gchunk * 4 * M * 8;                                      // gradient scratch
  (void)run;
  return b;
}

// ----------------------------------------------------------------------------
// integrator pieces
void fin(Ctx& c, int64_t nst, double* scale, bool do_scale, bool do_h) {
  StateScalars s = c.scalars(scale);
  const int nh = c.eng->ngx() + c.eng->ncb();
  c.launch(KC_FINALIZE, [&] {
    hipLaunchKernelGGL(k_finalize, dim3(cdiv(nst, 256)), dim3(256), 0, c.stream, nst, s, c.eng->ngx(), nh,
                       c.eng->raw_h_slots(), int(do_scale), int(do_h), c.dV);
  });
}

// streaming device copy (bytes a multiple of 16, both ends 16-byte aligned)
void device_copy(void* dst, const void* src, int64_t bytes, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return;
  hipLaunchKernelGGL(k_stream_copy, dim3(cdiv(n16, CP_TB * CP_U)), dim3(CP_TB), 0, st, (const cp_v4i*)src,
                     (cp_v4i*)dst, n16);
  HIPCHK(hipGetLastError());
}

// buffer b was rewritten by a kernel that leaves no kinetic partials
inline void touched(Ctx& c, int b) { c.kin_ready[b] = false; }

// fields and <H>_n of buffer b (its scale must be current); leaves T = D2x
void prepare(Ctx& c, int b) {
  if (c.kin_ready[b])
    c.eng->dens_sum(c, c.sb[b], c.sscale[b], c.nst);
  else
    c.eng->dens(c, c.sb[b], c.sscale[b], c.nst);
  c.eng->reduce_pot(c, !c.frozen);
  if (c.fric && !c.frozen) c.eng->friction(c, c.sb[b], c.sscale[b], c.nst);
  c.eng->lap1(c, c.sb[b], c.sscale[b], true, c.nst);
  fin(c, c.nst, c.sscale[b], false, true);
  c.fields_valid = true;
}

// what an F / CORR / FULL evaluation of buffer b needs: the fields, and the
// shift unless the engine's lap2 takes it itself
void prepare_eval(Ctx& c, int b) {
  if (!c.eng->self_shift()) {
    prepare(c, b);
    return;
  }
  c.eng->dens_sum(c, c.sb[b], c.sscale[b], c.nst);
  c.eng->reduce_pot(c, !c.frozen);
  if (c.fric && !c.frozen) c.eng->friction(c, c.sb[b], c.sscale[b], c.nst);
  c.fields_valid = true;
}

void norm_of(Ctx& c, int b) {
  PwDesc d;
  d.mode = PW_NORM;
  d.X = c.sb[b];
  d.nrm_part = c.nrm_part;
  c.eng->pointwise(c, d, c.nst);
  fin(c, c.nst, c.sscale[b], true, false);
}

void f_into(Ctx& c, int src, int dst) {
  L2Desc d;
  d.mode = L2_F;
  d.X = c.sb[src];
  d.T = c.T;
  d.scale = c.sscale[src];
  d.hshift = c.hshift;
  d.out = c.sb[dst];
  c.eng->lap2(c, d, c.nst);
  touched(c, dst);
}

// Taylor series sum_{k<=r} (-i tau)^k/k! (H - h)^k phi with H, h already
// prepared (fields, hshift).  t_ready: T already holds D2x of phi.  Writes
// into buffer acc and finalises its scale; psi_k is formed in place in pa.
void taylor_series(Ctx& c, int phi, int acc, int pa, double tau, bool t_ready) {
  const int r = c.run.taylor_order > 0 ? c.run.taylor_order : 5;
  for (int k = 1; k <= r; ++k) {
    const bool first = k == 1;
    const int in = first ? phi : pa;
    if (!first || !t_ready) c.eng->lap1(c, c.sb[in], first ? c.sscale[phi] : nullptr, false, c.nst);
    L2Desc d;
    d.mode = L2_TAYLOR;
    d.X = c.sb[in];
    d.T = c.T;
    d.scale = first ? c.sscale[phi] : nullptr;
    d.hshift = c.hshift;
    d.out = c.sb[pa];
    d.acc = c.sb[acc];
    d.init_acc = first ? 1 : 0;
    d.tay_re = 0.0;
    d.tay_im = -tau / k;  // (-i tau / k)
    d.nrm_part = (k == r) ? c.nrm_part : nullptr;
    c.eng->lap2(c, d, c.nst);
  }
  touched(c, pa);
  touched(c, acc);
  fin(c, c.nst, c.sscale[acc], true, false);
}

// One start-up step phi -> new buffer, by the Taylor predictor-corrector of
// Eq. Taylor-exp (H at the mid point, shifted operator H - <H>_n with <H>_n
// on the state the H is built from; mid point and result renormalised).
// Requires prepare(phi) done.  Returns the new buffer.
int taylor_step(Ctx& c, int phi, std::vector<int>& freeb) {
  require(freeb.size() >= 2, TDSLDA_EINVAL, "internal: not enough buffers for the start-up");
  int pa = freeb.back(); freeb.pop_back();
  int acc = freeb.back(); freeb.pop_back();
  taylor_series(c, phi, acc, pa, 0.5 * c.run.dt, true);  // mid-point state
  prepare(c, acc);                                        // fields and <H> at the mid point
  taylor_series(c, phi, acc, pa, c.run.dt, false);        // full step from phi
  freeb.push_back(pa);
  return acc;
}

void start(Ctx& c) {
  const int D = c.depth;
  std::vector<int> freeb;
  for (int b = 0; b <= D; ++b)
    if (b != c.phi) freeb.push_back(b);
  norm_of(c, c.phi);
  std::vector<int> hl;  // newest first
  if (c.run.selfstart == 0) {
    prepare(c, c.phi);
    int f0 = freeb.back();
    freeb.pop_back();
    f_into(c, c.phi, f0);
    hl.push_back(f0);
    while ((int)hl.size() < D) {
      int b = freeb.back();
      freeb.pop_back();
      device_copy(c.sb[b], c.sb[f0], int64_t(c.nst) * 2 * c.M * int64_t(c.esz), c.stream);
      touched(c, b);
      hl.push_back(b);
    }
  } else {
    // phi_0 .. phi_{D-1} by Taylor steps; history f(phi_j), newest first
    int cur = c.phi;
    for (int j = 0; j < D; ++j) {
      int nxt = -1;
      if (j < D - 1) {
        prepare(c, cur);
        nxt = taylor_step(c, cur, freeb);
      }
      prepare(c, cur);
      int fs = freeb.back();
      freeb.pop_back();
      f_into(c, cur, fs);
      hl.insert(hl.begin(), fs);
      if (nxt >= 0) {
        freeb.push_back(cur);
        cur = nxt;
        c.time += c.run.dt;
      }
    }
    c.phi = cur;
  }
  for (int j = 0; j < D; ++j) c.hist[j] = hl[j];
  c.started = true;
}

void abm(Ctx& c, int64_t nsteps) {
  if (!c.started) start(c);
  if (nsteps <= 0) return;
  const int D = c.depth;
  // predictor + partial corrector of the first step
  {
    PwDesc d;
    d.mode = PW_PRED;
    d.X = c.sb[c.phi];
    d.scale = c.sscale[c.phi];
    for (int j = 0; j < D; ++j) d.hist[j] = c.sb[c.hist[j]];
    d.cout = c.sb[c.hist[D - 1]];
    d.nrm_part = c.nrm_part;
    c.eng->pointwise(c, d, c.nst);
    fin(c, c.nst, c.sscale[c.phi], true, false);
    touched(c, c.phi);
    touched(c, c.hist[D - 1]);
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    // evaluation at the predicted state; corrector
    prepare_eval(c, c.phi);
    {
      L2Desc d;
      d.mode = L2_CORR;
      d.X = c.sb[c.phi];
      d.Xout = c.sb[c.phi];
      d.T = c.T;
      d.scale = c.sscale[c.phi];
      d.hshift = c.hshift;
      d.hist[0] = c.sb[c.hist[D - 1]];  // partial corrector c
      d.nrm_part = c.nrm_part;
      c.eng->lap2(c, d, c.nst);
      fin(c, c.nst, c.sscale[c.phi], true, false);
      c.kin_ready[c.phi] = c.eng->producer_kinetic();
    }
    // rotate: the slot of c becomes the slot of the new f
    {
      int freed = c.hist[D - 1];
      for (int j = D - 1; j > 0; --j) c.hist[j] = c.hist[j - 1];
      c.hist[0] = freed;
    }
    // evaluation at the corrected state
    prepare_eval(c, c.phi);
    L2Desc d;
    d.X = c.sb[c.phi];
    d.T = c.T;
    d.scale = c.sscale[c.phi];
    d.hshift = c.hshift;
    d.out = c.sb[c.hist[0]];
    if (s + 1 < nsteps) {
      d.mode = L2_FULL;
      d.Xout = c.sb[c.phi];
      for (int j = 1; j < D; ++j) d.hist[j] = c.sb[c.hist[j]];
      d.cout = c.sb[c.hist[D - 1]];
      d.nrm_part = c.nrm_part;
      c.eng->lap2(c, d, c.nst);
      fin(c, c.nst, c.sscale[c.phi], true, false);
      c.kin_ready[c.phi] = c.eng->producer_kinetic();
      touched(c, c.hist[D - 1]);
    } else {
      d.mode = L2_F;
      c.eng->lap2(c, d, c.nst);
    }
    touched(c, c.hist[0]);
    c.steps += 1;
    c.time += c.run.dt;
  }
}

// rho, tau, nu, j of the current states into the device fields; refresh
// the mean fields unless frozen.
void full_densities(Ctx& c) {
  const int b = c.phi;
  c.eng->dens(c, c.sb[b], c.sscale[b], c.nst);
  c.eng->reduce_pot(c, !c.frozen);
  if (!c.frozen) c.fields_valid = true;
  if (c.aslda) return;  // the ASLDA density pass builds tau and j of both spins
  for (int64_t n0 = 0; n0 < c.nst; n0 += c.gchunk) {
    const int64_t nch = std::min(c.gchunk, c.nst - n0);
    c.eng->grad(c, c.sb[b], c.sscale[b], n0, nch);
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL(k_grad_reduce, dim3(cdiv(c.M, 256)), dim3(256), 0, c.stream, nch, c.M, c.ainv,
                         c.gscratch, c.gscratch + nch * c.M, c.tau, c.jc, int(n0 == 0));
    });
  }
}

void energy(Ctx& c, double* out8) {  // out8[9]
  full_densities(c);
  if (c.aslda) {
    c.launch(KC_ENERGY, [&] {
      hipLaunchKernelGGL(k_energy_aslda, dim3(1), dim3(1024), 0, c.stream, c.M, c.rho, c.tau, c.nu, c.jc, c.delta,
                         c.vext, c.dext, c.dVe, c.eout);
    });
    double h[9];
    HIPCHK(hipMemcpyAsync(h, c.eout, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const double N = h[5];
    const double ef = 0.5 * std::pow(3.0 * kPi * kPi * N / c.vol, 2.0 / 3.0);
    for (int k = 0; k < 5; ++k) out8[k] = h[k];
    out8[5] = h[0] + h[1] + h[2] + h[3] + h[4] + h[6];
    out8[6] = N;
    out8[7] = 0.6 * N * ef;
    out8[8] = h[6];
    return;
  }
  c.launch(KC_ENERGY, [&] {
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, c.stream, c.M, c.rho, c.tau, c.nu, c.jc, c.delta,
                       c.vext, c.dext, c.fun.B, c.fun.functional == TDSLDA_FUNC_SLDA ? c.fun.A : 1.0,
                       int(c.fun.functional == TDSLDA_FUNC_SLDA), c.dVe, c.eout);
  });
  double h[7];
  HIPCHK(hipMemcpyAsync(h, c.eout, sizeof(h), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  const double N = h[5];
  const double ef = 0.5 * std::pow(3.0 * kPi * kPi * N / c.vol, 2.0 / 3.0);
  out8[0] = h[0];
  out8[1] = h[1];
  out8[2] = h[2];
  out8[3] = h[3];
  out8[4] = h[4];
  out8[5] = h[0] + h[1] + h[2] + h[3] + h[4] + h[6];
  out8[6] = N;
  out8[7] = 0.6 * N * ef;
  out8[8] = h[6];
}

// frozen (linear-mode) fields: hA = U + V_ext - mu, hD = Delta + Delta_ext
void set_frozen_fields(Ctx& c) {
  c.launch(KC_SETUP, [&] {
    if (c.esz == 16)
      hipLaunchKernelGGL((k_set_fields<double>), dim3(cdiv(c.M, 256)), dim3(256), 0, c.stream, c.M, c.U, c.delta,
                         c.vext, c.dext, c.fun.mu, (double*)c.hA, (cpx<double>*)c.hD);
    else
      hipLaunchKernelGGL((k_set_fields<float>), dim3(cdiv(c.M, 256)), dim3(256), 0, c.stream, c.M, c.U, c.delta,
                         c.vext, c.dext, c.fun.mu, (float*)c.hA, (cpx<float>*)c.hD);
  });
}

// the functional's own alpha (A; 1 for BdG), D2 alpha = 0, A_z = 0; the
// general operator is in use when the functional has A != 1
// ASLDA: A(p = 0) for both spins until the first field build
void reset_current_fields(Ctx& c) {
  const double a = c.aslda ? 1.094 : c.fun.functional == TDSLDA_FUNC_SLDA ? c.fun.A : 1.0;
  const int64_t nf = c.aslda ? 2 * c.M : c.M;  // field values ([spin][M] for ASLDA)
  c.launch(KC_SETUP, [&] {
    if (c.esz == 16)
      hipLaunchKernelGGL((k_fill_real<double>), dim3(cdiv(nf, 256)), dim3(256), 0, c.stream, nf, a, (double*)c.hAl);
    else
      hipLaunchKernelGGL((k_fill_real<float>), dim3(cdiv(nf, 256)), dim3(256), 0, c.stream, nf, a, (float*)c.hAl);
  });
  HIPCHK(hipMemsetAsync(c.hLa, 0, nf * c.esz / 2, c.stream));
  for (void* p : {c.hAx, c.hAy, c.hAz})
    if (p) HIPCHK(hipMemsetAsync(p, 0, nf * c.esz / 2, c.stream));
  c.gen = c.aslda || a != 1.0;
}

void after_load(Ctx& c) {
  for (bool& k : c.kin_ready) k = false;
  c.loaded = true;
  c.started = false;
  c.steps = 0;
  c.time = 0;
  c.have_ref = false;
  c.phi = 0;
  for (int j = 0; j < 5; ++j) c.hist[j] = j + 1;
  norm_of(c, c.phi);
  if (!c.frozen) {
    c.eng->dens(c, c.sb[c.phi], c.sscale[c.phi], c.nst);
    c.eng->reduce_pot(c, true);
    c.fields_valid = true;
  }
}

void set_weights(Ctx& c, int64_t n, const double* E_host) {
  if (E_host) HIPCHK(hipMemcpyAsync(c.E, E_host, n * 8, hipMemcpyHostToDevice, c.stream));
  c.launch(KC_SETUP, [&] {
    hipLaunchKernelGGL(k_weights, dim3(cdiv(n, 256)), dim3(256), 0, c.stream, n, c.E, c.fun.temperature, c.mult,
                       c.wu, c.wv);
  });
}

template <class F>
tdslda_status guard(tdslda_ctx* c, F&& f) {
  if (!c) return TDSLDA_EINVAL;
  try {
    c->err.clear();
    f();
    return TDSLDA_OK;
  } catch (const Fail& e) {
    c->err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return TDSLDA_ENOMEM;
  } catch (...) {
    c->err = "unknown error";
    return TDSLDA_EDEVICE;
  }
}

void check_lattice(const tdslda_lattice& lat) {
  if (lat.mode == TDSLDA_MODE_3D) {
    require(lat.nx > 0 && lat.ny > 0 && lat.nz > 0 && lat.nx % 2 == 0 && lat.ny % 2 == 0 && lat.nz % 2 == 0,
            TDSLDA_EINVAL, "lattice sizes must be positive and even");
    require(lat.dx > 0 && lat.dy > 0 && lat.dz > 0, TDSLDA_EINVAL, "lattice spacings must be positive");
  } else if (lat.mode == TDSLDA_MODE_Q1D) {
    require(lat.nz > 0 && lat.nz % 2 == 0 && lat.dz > 0, TDSLDA_EINVAL, "bad quasi-1D lattice");
    require(lat.lx_perp > 0 && lat.ly_perp > 0, TDSLDA_EINVAL, "quasi-1D needs the transverse box");
  } else if (lat.mode == TDSLDA_MODE_Q2D) {
    require(lat.nx > 0 && lat.ny > 0 && lat.nx % 2 == 0 && lat.ny % 2 == 0, TDSLDA_EINVAL,
            "quasi-2D lattice sizes must be positive and even");
    require(lat.nz > 0 && lat.nz % 2 == 0, TDSLDA_EINVAL, "quasi-2D needs an even number of k_z plane waves");
    require(lat.dx > 0 && lat.dy > 0 && lat.dz > 0, TDSLDA_EINVAL, "lattice spacings must be positive");
  } else {
    throw Fail{TDSLDA_EINVAL, "unknown lattice mode"};
  }
}

}  // namespace

// ============================================================================
// C ABI
extern "C" {

const char* tdslda_kernel_name(int k) { return (k >= 0 && k < KC_COUNT) ? kKernelNames[k] : nullptr; }

tdslda_status tdslda_device_copy(void* dst, const void* src, int64_t bytes, void* hip_stream) {
  if (!dst || !src || bytes < 0 || bytes % 16 || (uintptr_t(dst) | uintptr_t(src)) % 16) return TDSLDA_EINVAL;
  const uintptr_t d = uintptr_t(dst), s = uintptr_t(src);
  if (d < s + uint64_t(bytes) && s < d + uint64_t(bytes) && bytes > 0) return TDSLDA_EINVAL;
  if (bytes / 16 > int64_t(0x7fffffff) * CP_TB * CP_U) return TDSLDA_EINVAL;
  try {
    device_copy(dst, src, bytes, (hipStream_t)hip_stream);
    return TDSLDA_OK;
  } catch (const Fail& e) {
    return e.st;
  }
}

tdslda_status tdslda_device_read(const void* src, int64_t bytes, void* sink16, void* hip_stream) {
  if (!src || !sink16 || bytes < 0 || bytes % 16 || (uintptr_t(src) | uintptr_t(sink16)) % 16) return TDSLDA_EINVAL;
  if (bytes / 16 > int64_t(0x7fffffff) * RD_TB * RD_U) return TDSLDA_EINVAL;
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return TDSLDA_OK;
  hipLaunchKernelGGL(k_stream_read, dim3(cdiv(n16, RD_TB * RD_U)), dim3(RD_TB), 0, (hipStream_t)hip_stream,
                     (const cp_v4i*)src, (cp_v4i*)sink16, n16);
  if (hipGetLastError() != hipSuccess) return TDSLDA_EDEVICE;
  return TDSLDA_OK;
}

const char* tdslda_last_error(const tdslda_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

tdslda_status tdslda_memory_plan(const tdslda_lattice* lat, const tdslda_run* run, int64_t nstates,
                                 int64_t* bytes_out) {
  if (!lat || !run || !bytes_out || nstates < 0) return TDSLDA_EINVAL;
  try {
    check_lattice(*lat);
    auto eng = make_engine(*lat, run->precision);
    if (!eng) return TDSLDA_EINVAL;
    tdslda_ctx tmp;
    tmp.run = *run;
    set_scheme(tmp);
    const int64_t M = lat->mode == TDSLDA_MODE_3D    ? int64_t(lat->nx) * lat->ny * lat->nz
                      : lat->mode == TDSLDA_MODE_Q2D ? int64_t(lat->nx) * lat->ny
                                                     : lat->nz;
    (void)M;
    *bytes_out = memory_bytes(*lat, *run, nstates, eng.get(), tmp.depth, std::min<int64_t>(nstates, 64));
    return TDSLDA_OK;
  } catch (...) {
    return TDSLDA_EINVAL;
  }
}

tdslda_status tdslda_create(const tdslda_lattice* lat, const tdslda_functional* fun, const tdslda_run* run,
                            int64_t capacity, tdslda_ctx** out) {
  if (!lat || !fun || !run || !out || capacity <= 0) return TDSLDA_EINVAL;
  *out = nullptr;
  tdslda_ctx* c = new (std::nothrow) tdslda_ctx();
  if (!c) return TDSLDA_ENOMEM;
  tdslda_status st = guard(c, [&] {
    check_lattice(*lat);
    require(run->precision == TDSLDA_FP64 || run->precision == TDSLDA_FP32_MIXED, TDSLDA_EINVAL,
            "unknown precision");
    require(fun->functional == TDSLDA_FUNC_SLDA || fun->functional == TDSLDA_FUNC_BDG ||
                fun->functional == TDSLDA_FUNC_ASLDA,
            TDSLDA_EINVAL, "unknown functional");
    require(fun->functional != TDSLDA_FUNC_ASLDA || lat->mode == TDSLDA_MODE_Q1D || lat->mode == TDSLDA_MODE_3D,
            TDSLDA_EINVAL, "the spin-imbalanced ASLDA functional is built for the quasi-1D and full-3D kernel sets");
    require(fun->functional != TDSLDA_FUNC_ASLDA || (std::isfinite(fun->mu) && std::isfinite(fun->mu_b)),
            TDSLDA_EINVAL, "mu_a and mu_b must be finite");
    require(fun->functional != TDSLDA_FUNC_SLDA || (std::isfinite(fun->A) && fun->A > 0), TDSLDA_EINVAL,
            "A must be positive");
    require(std::isfinite(run->dt) && run->dt != 0.0, TDSLDA_EINVAL, "dt must be finite and non-zero");
    c->lat = *lat;
    c->fun = *fun;
    c->run = *run;
    c->q1d = lat->mode == TDSLDA_MODE_Q1D;
    c->q2d = lat->mode == TDSLDA_MODE_Q2D;
    c->aslda = fun->functional == TDSLDA_FUNC_ASLDA;
    if (c->aslda) c->fun.C = -11.11;  // C(p) of the ASLDA parametrisation
    require(!c->q2d || fun->functional != TDSLDA_FUNC_SLDA || fun->A == 1.0, TDSLDA_EINVAL,
            "the quasi-2D kernel set is built for the A = 1 functional");
    c->stream = (hipStream_t)run->hip_stream;
    set_scheme(*c);
    c->eng = make_engine(*lat, run->precision);
    require(c->eng != nullptr, TDSLDA_EINVAL, "unsupported lattice shape");
    c->esz = c->eng->elem_size();
    if (c->q1d) {
      c->M = lat->nz;
      c->dV = lat->dz;
      c->ainv = 1.0 / (lat->lx_perp * lat->ly_perp);
      c->dVe = lat->dz * lat->lx_perp * lat->ly_perp;
      c->vol = lat->nz * lat->dz * lat->lx_perp * lat->ly_perp;
    } else if (c->q2d) {
      const double Lz = lat->nz * lat->dz;
      c->M = int64_t(lat->nx) * lat->ny;
      c->dV = lat->dx * lat->dy;
      c->ainv = 1.0 / Lz;
      c->dVe = c->dV * Lz;
      c->vol = c->M * c->dVe;
    } else {
      c->M = int64_t(lat->nx) * lat->ny * lat->nz;
      c->dV = lat->dx * lat->dy * lat->dz;
      c->ainv = 1.0;
      c->dVe = c->dV;
      c->vol = c->M * c->dV;
    }
    require(lat->mode != TDSLDA_MODE_3D || capacity <= 65535, TDSLDA_EINVAL,
            "full-3D contexts hold at most 65535 states (one grid row per state)");
    c->cap = capacity;
    const int64_t M = c->M;
    const size_t S = size_t(2 * M) * c->esz;
    for (int b = 0; b <= c->depth; ++b) c->sb[b] = c->dalloc(S * capacity);
    if (!c->q2d) c->T = c->dalloc(S * capacity);  // the quasi-2D passes need no intermediate
    for (int b = 0; b <= c->depth; ++b) c->sscale[b] = (double*)c->dalloc(8 * capacity);
    c->wu = (double*)c->dalloc(8 * capacity);
    c->wv = (double*)c->dalloc(8 * capacity);
    c->E = (double*)c->dalloc(8 * capacity);
    c->kperp2 = (double*)c->dalloc(8 * capacity);
    HIPCHK(hipMemsetAsync(c->kperp2, 0, 8 * capacity, c->stream));
    c->mult = (double*)c->dalloc(8 * capacity);
    hipLaunchKernelGGL(k_fill_real<double>, dim3(cdiv(capacity, 256)), dim3(256), 0, c->stream, capacity, 1.0,
                       c->mult);
    HIPCHK(hipGetLastError());
    c->hshift = (double*)c->dalloc(8 * capacity);
    c->nrm_stride = c->eng->ngx();
    c->h_stride = c->eng->ngx() + c->eng->ncb();
    c->nrm_part = (double*)c->dalloc(8 * capacity * c->nrm_stride);
    c->h_part = (double*)c->dalloc(8 * capacity * c->h_stride);
    c->nsg_max = int(cdiv(capacity, c->eng->group()));
    const int ncomp_part = c->aslda ? (c->q1d ? 8 : 12) : c->q1d ? 4 : 3;  // density partials per group
    c->dens_part = (double*)c->dalloc(size_t(c->nsg_max) * ncomp_part * M * 8);
    const int64_t ns = c->aslda ? 2 : 1;  // spin-resolved densities and fields
    c->rho = (double*)c->dalloc(8 * M * ns);
    c->nu = (double*)c->dalloc(16 * M);
    c->tau = (double*)c->dalloc(8 * M * ns);
    c->jc = (double*)c->dalloc(24 * M * ns);  // [spin][3][M] for ASLDA
    c->U = (double*)c->dalloc(8 * M * ns);
    c->delta = (double*)c->dalloc(16 * M);
    c->vext = (double*)c->dalloc(8 * M);
    c->lam = (double*)c->dalloc(8 * M);
    c->theta = (double*)c->dalloc(8 * M);
    c->dext = (double*)c->dalloc(16 * M);
    HIPCHK(hipMemsetAsync(c->dext, 0, 16 * M, c->stream));
    c->hA = c->dalloc(M * ns * c->esz / 2);
    c->hD = c->dalloc(M * c->esz);
    c->hAl = c->dalloc(M * ns * c->esz / 2);
    c->hLa = c->dalloc(M * ns * c->esz / 2);
    c->hAz = c->dalloc(M * ns * c->esz / 2);
    if (lat->mode == TDSLDA_MODE_3D) {
      c->hAx = c->dalloc(M * ns * c->esz / 2);
      c->hAy = c->dalloc(M * ns * c->esz / 2);
      if (c->aslda) {  // the D2 circulants of the three axes, for the Laplacians of alpha_s
        const auto cx = spectral_d2_circulant(lat->nx, lat->dx), cy = spectral_d2_circulant(lat->ny, lat->dy),
                   cz = spectral_d2_circulant(lat->nz, lat->dz);
        c->circ = (double*)c->dalloc(8 * (cx.size() + cy.size() + cz.size()));
        HIPCHK(hipMemcpyAsync(c->circ, cx.data(), 8 * cx.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->circ + cx.size(), cy.data(), 8 * cy.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->circ + cx.size() + cy.size(), cz.data(), 8 * cz.size(), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));  // the host vectors go out of scope
      }
      c->jpart = (double*)c->dalloc(size_t(c->nsg_max) * 3 * M * 8);
    }
    reset_current_fields(*c);
    HIPCHK(hipMemsetAsync(c->vext, 0, 8 * M, c->stream));
    HIPCHK(hipMemsetAsync(c->lam, 0, 8 * M, c->stream));
    c->gchunk = std::min<int64_t>(capacity, 64);
    c->gscratch = (double*)c->dalloc(size_t(c->gchunk) * 4 * M * 8);
    c->eout = (double*)c->dalloc(16 * sizeof(double));  // energy terms (up to 9)
    c->dflag = (int*)c->dalloc(16);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
  if (st != TDSLDA_OK) {
    // report through a stderr line: the context cannot outlive the failure
    std::fprintf(stderr, "tdslda_create: %s\n", c->err.c_str());
    delete c;
    return st;
  }
  *out = c;
  return TDSLDA_OK;
}

tdslda_status tdslda_destroy(tdslda_ctx* ctx) {
  if (!ctx) return TDSLDA_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return TDSLDA_OK;
}

tdslda_status tdslda_set_external(tdslda_ctx* c, const double* vext, const double* dext_reim,
                                  int freeze_regulator) {
  return guard(c, [&] {
    require(vext != nullptr, TDSLDA_EINVAL, "vext is NULL");
    if (dext_reim)
      for (int64_t i = 0; i < 2 * c->M; ++i)
        require(std::isfinite(dext_reim[i]), TDSLDA_EINVAL, "Delta_ext is not finite");
    HIPCHK(hipMemcpyAsync(c->vext, vext, 8 * c->M, hipMemcpyHostToDevice, c->stream));
    c->dext_on = false;
    if (dext_reim) {
      HIPCHK(hipMemcpyAsync(c->dext, dext_reim, 16 * c->M, hipMemcpyHostToDevice, c->stream));
      for (int64_t i = 0; i < 2 * c->M; ++i) c->dext_on = c->dext_on || dext_reim[i] != 0.0;
    } else {
      HIPCHK(hipMemsetAsync(c->dext, 0, 16 * c->M, c->stream));
    }
    c->have_ref = false;
    if (freeze_regulator) {
      HIPCHK(hipMemsetAsync(c->dflag, 0, 4, c->stream));
      c->launch(KC_SETUP, [&] {
        // ASLDA: the spin averages A_+ = A(p = 0), mu_+ (Eq. Creg)
        hipLaunchKernelGGL(k_lambda, dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M, c->vext,
                           c->aslda ? 0.5 * (c->fun.mu + c->fun.mu_b) : c->fun.mu, c->fun.ec_reg,
                           c->aslda ? 1.094 : c->fun.functional == TDSLDA_FUNC_SLDA ? c->fun.A : 1.0, c->lam,
                           c->dflag);
      });
      int bad = 0;
      HIPCHK(hipMemcpyAsync(&bad, c->dflag, 4, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      require(!bad, TDSLDA_EINVAL, "E_c below the local band bottom in Lambda_c");
    }
    if (c->loaded && !c->frozen) {
      c->eng->dens(*c, c->sb[c->phi], c->sscale[c->phi], c->nst);
      c->eng->reduce_pot(*c, true);
    }
    if (c->frozen) set_frozen_fields(*c);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_regulator(tdslda_ctx* c, const double* lam) {
  return guard(c, [&] {
    require(lam != nullptr, TDSLDA_EINVAL, "lam is NULL");
    HIPCHK(hipMemcpyAsync(c->lam, lam, 8 * c->M, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

static void load_common(tdslda_ctx* c, int64_t n, const double* E, const double* kperp2) {
  require(n > 0 && n <= c->cap, TDSLDA_EINVAL, "state count out of range [1, capacity]");
  require(E != nullptr, TDSLDA_EINVAL, "E is NULL");
  if (c->q1d || c->q2d) {
    require(kperp2 != nullptr, TDSLDA_EINVAL, c->q1d ? "quasi-1D states need kperp2" : "quasi-2D states need k_z^2");
    HIPCHK(hipMemcpyAsync(c->kperp2, kperp2, 8 * n, hipMemcpyHostToDevice, c->stream));
  }
  hipLaunchKernelGGL(k_fill_real<double>, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, 1.0, c->mult);
  HIPCHK(hipGetLastError());
  c->nst = n;
  set_weights(*c, n, E);
}

tdslda_status tdslda_load_states(tdslda_ctx* c, int64_t n, const double* uv, const double* E,
                                 const double* kperp2) {
  return guard(c, [&] {
    require(uv != nullptr, TDSLDA_EINVAL, "uv is NULL");
    load_common(c, n, E, kperp2);
    const int64_t per = 2 * c->M;  // complex elements per state
    if (c->esz == 16) {
      HIPCHK(hipMemcpyAsync(c->sb[0], uv, size_t(n) * per * 16, hipMemcpyHostToDevice, c->stream));
    } else {
      // stage through the gradient scratch (gchunk states of FP64) and round
      for (int64_t n0 = 0; n0 < n; n0 += c->gchunk) {
        const int64_t k = std::min(c->gchunk, n - n0);
        HIPCHK(hipMemcpyAsync(c->gscratch, uv + n0 * per * 2, size_t(k) * per * 16, hipMemcpyHostToDevice, c->stream));
        c->launch(KC_SETUP, [&] {
          hipLaunchKernelGGL((k_convert_in<float>), dim3(cdiv(k * per, 256)), dim3(256), 0, c->stream, k * per,
                             (const cpx<double>*)c->gscratch, (cpx<float>*)c->sb[0] + n0 * per);
        });
      }
    }
    after_load(*c);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_load_states_device(tdslda_ctx* c, int64_t n, const void* uv_dev, const double* E,
                                        const double* kperp2) {
  return guard(c, [&] {
    require(uv_dev != nullptr, TDSLDA_EINVAL, "uv_dev is NULL");
    load_common(c, n, E, kperp2);
    HIPCHK(hipMemcpyAsync(c->sb[0], uv_dev, size_t(n) * 2 * c->M * c->esz, hipMemcpyDeviceToDevice, c->stream));
    after_load(*c);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_multiplicity(tdslda_ctx* c, int64_t n, const double* mult) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states first");
    require(!c->started, TDSLDA_EORDER, "set the multiplicities before the first step");
    require(mult != nullptr && n == c->nst, TDSLDA_EINVAL, "give one multiplicity per loaded state");
    for (int64_t i = 0; i < n; ++i)
      require(std::isfinite(mult[i]) && mult[i] > 0.0, TDSLDA_EINVAL, "multiplicities must be finite, > 0");
    HIPCHK(hipMemcpyAsync(c->mult, mult, 8 * n, hipMemcpyHostToDevice, c->stream));
    set_weights(*c, n, nullptr);
    after_load(*c);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_init_plane_waves(tdslda_ctx* c, int64_t n, const int32_t* kidx, double u0, double delta0) {
  return guard(c, [&] {
    require(!c->q1d, TDSLDA_EINVAL, "plane-wave start is a 3D and quasi-2D option");
    const int64_t nout = c->aslda ? 2 * n : n;  // ASLDA: both branches of every momentum
    require(kidx != nullptr && n > 0 && nout <= c->cap, TDSLDA_EINVAL, "bad plane-wave list");
    require(delta0 > 0, TDSLDA_EINVAL, "delta0 must be > 0");
    const int zmax = c->q2d ? c->lat.nz / 2 + 1 : c->lat.nz;  // quasi-2D: |k_z| classes 0 .. nz/2
    for (int64_t i = 0; i < n; ++i) {
      require(kidx[3 * i] >= 0 && kidx[3 * i] < c->lat.nx && kidx[3 * i + 1] >= 0 && kidx[3 * i + 1] < c->lat.ny &&
                  kidx[3 * i + 2] >= 0 && kidx[3 * i + 2] < zmax,
              TDSLDA_EINVAL, "k index out of range");
    }
    if (c->kidx_cap < n) {
      c->kidx_dev = (int32_t*)c->dalloc(size_t(n) * 12);
      c->kidx_cap = n;
    }
    HIPCHK(hipMemcpyAsync(c->kidx_dev, kidx, size_t(n) * 12, hipMemcpyHostToDevice, c->stream));
    c->nst = nout;
    const double kx = 2 * kPi / (c->lat.nx * c->lat.dx), ky = 2 * kPi / (c->lat.ny * c->lat.dy),
                 kz = 2 * kPi / (c->lat.nz * c->lat.dz);
    if (c->q2d) {
      const double isa = 1.0 / std::sqrt(c->M * c->dV);  // 2D normalisation (1/L_z is in the densities)
      c->launch(KC_SETUP, [&] {
        if (c->esz == 16)
          hipLaunchKernelGGL((k_q2_plane_waves<double>), dim3(cdiv(c->M, 256), state_rows(n)), dim3(256), 0, c->stream, c->M, n,
                             c->lat.nx, c->lat.ny, c->lat.nz, c->kidx_dev, u0 - c->fun.mu, delta0, kx, ky, kz, isa,
                             (cpx<double>*)c->sb[0], c->E, c->kperp2, c->mult);
        else
          hipLaunchKernelGGL((k_q2_plane_waves<float>), dim3(cdiv(c->M, 256), state_rows(n)), dim3(256), 0, c->stream, c->M, n,
                             c->lat.nx, c->lat.ny, c->lat.nz, c->kidx_dev, u0 - c->fun.mu, delta0, kx, ky, kz, isa,
                             (cpx<float>*)c->sb[0], c->E, c->kperp2, c->mult);
      });
      set_weights(*c, n, nullptr);
      after_load(*c);
      HIPCHK(hipStreamSynchronize(c->stream));
      return;
    }
    const double isv = 1.0 / std::sqrt(c->vol);
    const double mubar = c->aslda ? 0.5 * (c->fun.mu + c->fun.mu_b) : c->fun.mu;
    const double dsh = c->aslda ? -0.5 * (c->fun.mu - c->fun.mu_b) : 0.0;
    c->launch(KC_SETUP, [&] {
      if (c->esz == 16)
        hipLaunchKernelGGL((k_plane_waves<double>), dim3(cdiv(c->M, 256), state_rows(nout)), dim3(256), 0, c->stream,
                           c->M, nout, c->lat.nx, c->lat.ny, c->lat.nz, c->kidx_dev, u0 - mubar, delta0, kx, ky, kz,
                           isv, (cpx<double>*)c->sb[0], c->E, int(c->aslda), dsh);
      else
        hipLaunchKernelGGL((k_plane_waves<float>), dim3(cdiv(c->M, 256), state_rows(nout)), dim3(256), 0, c->stream,
                           c->M, nout, c->lat.nx, c->lat.ny, c->lat.nz, c->kidx_dev, u0 - mubar, delta0, kx, ky, kz,
                           isv, (cpx<float>*)c->sb[0], c->E, int(c->aslda), dsh);
    });
    hipLaunchKernelGGL(k_fill_real<double>, dim3(cdiv(nout, 256)), dim3(256), 0, c->stream, nout, 1.0, c->mult);
    HIPCHK(hipGetLastError());
    set_weights(*c, nout, nullptr);
    after_load(*c);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_imprint_vortices(tdslda_ctx* c, int nv, const double* xyq) {
  return guard(c, [&] {
    require(!c->q1d, TDSLDA_EINVAL, "vortex imprint is a 3D and quasi-2D option");
    require(c->loaded, TDSLDA_EORDER, "load states first");
    require(nv > 0 && nv <= 64 && xyq, TDSLDA_EINVAL, "bad vortex list");
    double* buf = c->gscratch;
    HIPCHK(hipMemcpyAsync(buf, xyq, nv * 3 * 8, hipMemcpyHostToDevice, c->stream));
    c->launch(KC_SETUP, [&] {
      hipLaunchKernelGGL(k_vortex_phase, dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M, c->lat.nx,
                         c->lat.ny, c->q2d ? 1 : c->lat.nz, c->lat.dx, c->lat.dy, nv, buf, c->theta);
    });
    c->launch(KC_SETUP, [&] {
      if (c->esz == 16)
        hipLaunchKernelGGL((k_imprint<double>), dim3(cdiv(c->M, 256), state_rows(c->nst)), dim3(256), 0, c->stream, c->M,
                           c->nst, c->theta, (cpx<double>*)c->sb[c->phi]);
      else
        hipLaunchKernelGGL((k_imprint<float>), dim3(cdiv(c->M, 256), state_rows(c->nst)), dim3(256), 0, c->stream, c->M,
                           c->nst, c->theta, (cpx<float>*)c->sb[c->phi]);
    });
    // a new initial state: restart the integrator from it
    touched(*c, c->phi);
    c->started = false;
    c->steps = 0;
    c->time = 0;
    c->have_ref = false;
    norm_of(*c, c->phi);
    if (!c->frozen) {
      c->eng->dens(*c, c->sb[c->phi], c->sscale[c->phi], c->nst);
      c->eng->reduce_pot(*c, true);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_fields(tdslda_ctx* c, const double* U, const double* delta_reim) {
  return guard(c, [&] {
    if (!U && !delta_reim) {
      c->frozen = false;
      c->fields_valid = false;
      reset_current_fields(*c);
      if (c->loaded) {
        c->eng->dens(*c, c->sb[c->phi], c->sscale[c->phi], c->nst);
        c->eng->reduce_pot(*c, true);
        c->fields_valid = true;
      }
      HIPCHK(hipStreamSynchronize(c->stream));
      return;
    }
    require(U && delta_reim, TDSLDA_EINVAL, "give both U and Delta, or neither");
    require(!c->aslda, TDSLDA_EINVAL, "linear mode is not built for the ASLDA functional");
    HIPCHK(hipMemcpyAsync(c->U, U, 8 * c->M, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->delta, delta_reim, 16 * c->M, hipMemcpyHostToDevice, c->stream));
    set_frozen_fields(*c);
    c->frozen = true;
    c->fields_valid = true;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_densities(tdslda_ctx* c, double* rho, double* tau, double* nu_reim, double* j) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states first");
    require(!c->aslda, TDSLDA_EINVAL, "an ASLDA context has spin-resolved densities (tdslda_densities_spin)");
    full_densities(*c);
    if (rho) HIPCHK(hipMemcpyAsync(rho, c->rho, 8 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (tau) HIPCHK(hipMemcpyAsync(tau, c->tau, 8 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (nu_reim) HIPCHK(hipMemcpyAsync(nu_reim, c->nu, 16 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (j) HIPCHK(hipMemcpyAsync(j, c->jc, 24 * c->M, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_densities_spin(tdslda_ctx* c, double* rho, double* tau, double* nu_reim, double* j) {
  return guard(c, [&] {
    require(c->aslda, TDSLDA_EINVAL, "not an ASLDA context");
    require(c->loaded, TDSLDA_EORDER, "load states first");
    full_densities(*c);
    if (rho) HIPCHK(hipMemcpyAsync(rho, c->rho, 16 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (tau) HIPCHK(hipMemcpyAsync(tau, c->tau, 16 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (nu_reim) HIPCHK(hipMemcpyAsync(nu_reim, c->nu, 16 * c->M, hipMemcpyDeviceToHost, c->stream));
    if (j) HIPCHK(hipMemcpyAsync(j, c->jc, 48 * c->M, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_get_fields(tdslda_ctx* c, double* U, double* delta_reim) {
  return guard(c, [&] {
    require(c->fields_valid, TDSLDA_EORDER, "no fields yet");
    if (U) HIPCHK(hipMemcpyAsync(U, c->U, 8 * c->M * (c->aslda ? 2 : 1), hipMemcpyDeviceToHost, c->stream));
    if (delta_reim) HIPCHK(hipMemcpyAsync(delta_reim, c->delta, 16 * c->M, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_apply_hbdg(tdslda_ctx* c, const void* in_dev, void* out_dev, int64_t n) {
  return guard(c, [&] {
    require(in_dev && out_dev && in_dev != out_dev, TDSLDA_EINVAL, "bad in/out pointers");
    require(n > 0 && n <= c->cap, TDSLDA_EINVAL, "n out of range");
    require(c->fields_valid, TDSLDA_EORDER, "no fields yet (load states or set fields)");
    c->eng->lap1(*c, in_dev, nullptr, false, n);
    L2Desc d;
    d.mode = L2_H;
    d.X = in_dev;
    d.T = c->T;
    d.out = out_dev;
    c->eng->lap2(*c, d, n);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_current_fields(tdslda_ctx* c, const double* alpha, const double* avec) {
  const double* az = avec;
  return guard(c, [&] {
    if (!alpha && !az) {
      reset_current_fields(*c);
      HIPCHK(hipStreamSynchronize(c->stream));
      return;
    }
    require(!c->q2d, TDSLDA_EINVAL, "the general operator is not built for the quasi-2D kernel set");
    require(!c->aslda, TDSLDA_EINVAL, "the ASLDA functional builds its own alpha and A fields");
    require(c->frozen, TDSLDA_EORDER, "freeze the fields (tdslda_set_fields) first");
    const int ncomp = c->q1d ? 1 : 3;  // quasi-1D: A_z only; 3D: A_x, A_y, A_z
    for (int64_t i = 0; i < c->M; ++i)
      require(!alpha || (std::isfinite(alpha[i]) && alpha[i] > 0.0), TDSLDA_EINVAL, "alpha must be finite, > 0");
    for (int64_t i = 0; az && i < ncomp * c->M; ++i) require(std::isfinite(az[i]), TDSLDA_EINVAL, "A must be finite");
    reset_current_fields(*c);
    if (!c->q1d) {
      // staging in the gradient scratch (>= 4 M doubles): alpha, then each A_d
      const auto cx = spectral_d2_circulant(c->lat.nx, c->lat.dx), cy = spectral_d2_circulant(c->lat.ny, c->lat.dy),
                 cz = spectral_d2_circulant(c->lat.nz, c->lat.dz);
      if (alpha) {
        double* st = c->gscratch;
        double* cc = st + c->M;  // circulants after the field
        HIPCHK(hipMemcpyAsync(st, alpha, 8 * c->M, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(cc, cx.data(), 8 * cx.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(cc + cx.size(), cy.data(), 8 * cy.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(cc + cx.size() + cy.size(), cz.data(), 8 * cz.size(), hipMemcpyHostToDevice, c->stream));
        c->launch(KC_SETUP, [&] {
          if (c->esz == 16)
            hipLaunchKernelGGL((k_field_lap3d<double>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->lat.nx,
                               c->lat.ny, c->lat.nz, st, cc, cc + cx.size(), cc + cx.size() + cy.size(),
                               (double*)c->hAl, (double*)c->hLa);
          else
            hipLaunchKernelGGL((k_field_lap3d<float>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->lat.nx,
                               c->lat.ny, c->lat.nz, st, cc, cc + cx.size(), cc + cx.size() + cy.size(),
                               (float*)c->hAl, (float*)c->hLa);
        });
        HIPCHK(hipStreamSynchronize(c->stream));
      }
      if (az) {
        void* dst[3] = {c->hAx, c->hAy, c->hAz};
        for (int d = 0; d < 3; ++d) {
          HIPCHK(hipMemcpyAsync(c->gscratch, az + d * c->M, 8 * c->M, hipMemcpyHostToDevice, c->stream));
          c->launch(KC_SETUP, [&] {
            if (c->esz == 16)
              hipLaunchKernelGGL((k_convert_real<double>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M,
                                 c->gscratch, (double*)dst[d]);
            else
              hipLaunchKernelGGL((k_convert_real<float>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M,
                                 c->gscratch, (float*)dst[d]);
          });
          HIPCHK(hipStreamSynchronize(c->stream));
        }
      }
      c->gen = true;
      HIPCHK(hipStreamSynchronize(c->stream));
      return;
    }
    // quasi-1D: staging in the gradient scratch (>= 2 M doubles): alpha, A_z
    if (alpha) {
      HIPCHK(hipMemcpyAsync(c->gscratch, alpha, 8 * c->M, hipMemcpyHostToDevice, c->stream));
      c->launch(KC_SETUP, [&] {
        if (c->esz == 16)
          hipLaunchKernelGGL((k_field_d2<double>), dim3(1), dim3(256), 0, c->stream, int(c->M), c->lat.dz, c->gscratch,
                             (double*)c->hAl, (double*)c->hLa);
        else
          hipLaunchKernelGGL((k_field_d2<float>), dim3(1), dim3(256), 0, c->stream, int(c->M), c->lat.dz, c->gscratch,
                             (float*)c->hAl, (float*)c->hLa);
      });
    }
    if (az) {
      HIPCHK(hipMemcpyAsync(c->gscratch + c->M, az, 8 * c->M, hipMemcpyHostToDevice, c->stream));
      c->launch(KC_SETUP, [&] {
        if (c->esz == 16)
          hipLaunchKernelGGL((k_convert_real<double>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M,
                             c->gscratch + c->M, (double*)c->hAz);
        else
          hipLaunchKernelGGL((k_convert_real<float>), dim3(cdiv(c->M, 256)), dim3(256), 0, c->stream, c->M,
                             c->gscratch + c->M, (float*)c->hAz);
      });
    }
    c->gen = true;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_friction(tdslda_ctx* c, double alpha, double beta, double gamma, double rho0,
                                  double N_req) {
  return guard(c, [&] {
    require(!c->gen, TDSLDA_EINVAL, "quantum friction is built for the A = 1 operator");
    require(!c->q2d, TDSLDA_EINVAL, "quantum friction is not built for the quasi-2D kernel set");
    require(!c->aslda, TDSLDA_EINVAL, "quantum friction is not built for the ASLDA functional");
    require(std::isfinite(alpha) && std::isfinite(beta) && std::isfinite(gamma) && std::isfinite(N_req) &&
                std::isfinite(rho0) && rho0 > 0.0,
            TDSLDA_EINVAL, "friction parameters must be finite, rho0 > 0");
    c->f_alpha = alpha;
    c->f_beta = beta;
    c->f_gamma = gamma;
    c->f_rho0 = rho0;
    c->f_Nreq = N_req > 0.0 ? N_req : 0.0;
    c->fric = alpha != 0.0 || beta != 0.0 || (gamma != 0.0 && N_req > 0.0);
    if (c->fric && !c->fric_part) {
      const int64_t ng = cdiv(c->cap, c->eng->group());
      c->fric_part = (double*)c->dalloc(sizeof(double) * 3 * size_t(ng) * c->M);
      c->fric_j = (double*)c->dalloc(sizeof(double) * (c->q1d ? 1 : 3) * c->M);
      c->fric_bp = (double*)c->dalloc(sizeof(double) * 2 * c->M);
      if (!c->q1d) {
        c->fric_div = (double*)c->dalloc(sizeof(double) * c->M);
        c->fric_N = (double*)c->dalloc(sizeof(double) * 2);
      }
    }
  });
}

tdslda_status tdslda_abm_step(tdslda_ctx* c, int64_t nsteps) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "abm_step before any state load");
    require(nsteps >= 0, TDSLDA_EINVAL, "nsteps < 0");
    abm(*c, nsteps);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_abm_graph(tdslda_ctx* c, int64_t nsteps, double graph_ms[2]) {
  return guard(c, [&] {
    require(c->loaded && c->started, TDSLDA_EORDER, "abm_graph needs a started integrator (call abm_step first)");
    require(!c->prof, TDSLDA_EORDER, "switch profiling off before recording a graph");
    require(nsteps >= 0, TDSLDA_EINVAL, "nsteps < 0");
    if (nsteps == 0) return;
    HIPCHK(hipStreamSynchronize(c->stream));
    // the previous call's graph has completed (its launch synchronised)
    c->release_graph();
    hipStream_t user = c->stream, cs = c->stream;
    if (cs == nullptr) {  // capture needs a real stream: the context's private one
      if (!c->graph_stream) HIPCHK(hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking));
      cs = c->graph_stream;
    }
    c->stream = cs;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    // recording runs abm() on the host, which advances the integrator's
    // bookkeeping (buffer roles, kinetic-partial flags, step count, time)
    // without touching device memory: keep a copy to restore if the graph
    // never runs
    const int phi0 = c->phi;
    int hist0[5];
    bool kin0[6];
    std::copy(c->hist, c->hist + 5, hist0);
    std::copy(c->kin_ready, c->kin_ready + 6, kin0);
    const int64_t steps0 = c->steps;
    const double time0 = c->time;
    const bool fv0 = c->fields_valid;
    bool launched = false;
    auto cleanup = [&] {
      if (ge) (void)hipGraphExecDestroy(ge);
      if (g) (void)hipGraphDestroy(g);
      c->stream = user;
    };
    try {
      const auto t0 = std::chrono::steady_clock::now();
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        abm(*c, nsteps);
      } catch (...) {
        (void)hipStreamEndCapture(cs, &g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(cs, &g));
      HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      const auto t1 = std::chrono::steady_clock::now();
      launched = true;
      HIPCHK(hipGraphLaunch(ge, cs));
      HIPCHK(hipStreamSynchronize(cs));
      const auto t2 = std::chrono::steady_clock::now();
      if (graph_ms) {
        graph_ms[0] = std::chrono::duration<double, std::milli>(t1 - t0).count();
        graph_ms[1] = std::chrono::duration<double, std::milli>(t2 - t1).count();
      }
    } catch (...) {
      cleanup();
      if (!launched) {
        // nothing ran on the device: the context is as before the call
        c->phi = phi0;
        std::copy(hist0, hist0 + 5, c->hist);
        std::copy(kin0, kin0 + 6, c->kin_ready);
        c->steps = steps0;
        c->time = time0;
        c->fields_valid = fv0;
      } else {
        // the launch failed part-way: the buffers no longer match any
        // bookkeeping, so the states must be loaded again
        c->loaded = false;
        c->started = false;
      }
      throw;
    }
    // keep the executed graph until the next call or the context's end
    c->graph = g;
    c->graph_exec = ge;
    c->stream = user;
  });
}

tdslda_status tdslda_autotune(tdslda_ctx* c, int* nclasses, int32_t choice[4], double ms[4]) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states before tuning");
    const int k = c->eng->autotune(*c, choice, ms);
    if (nclasses) *nclasses = k;
    // the trial launches overwrote the scratch <H> slots: the next
    // evaluation rebuilds them with the full density pass
    if (k > 0)
      for (bool& r : c->kin_ready) r = false;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_q1d_count(const tdslda_lattice* lat, int nprob, const double* kperp2, const double* hfield,
                               const double* delta, double ecut, int32_t* counts, int64_t* total) {
  if (!lat || !kperp2 || !hfield || !delta || nprob <= 0 || lat->mode != TDSLDA_MODE_Q1D) return TDSLDA_EINVAL;
  try {
    check_lattice(*lat);
    const int64_t t = q1d_static(nullptr, lat->nz, lat->dz, nprob, kperp2, hfield, delta, ecut, counts, nullptr, 0,
                                 nullptr, nullptr, 0);
    if (total) *total = t;
    return TDSLDA_OK;
  } catch (const Fail& e) {
    std::fprintf(stderr, "tdslda_q1d_count: %s\n", e.msg.c_str());
    return e.st;
  } catch (...) {
    return TDSLDA_EDEVICE;
  }
}

tdslda_status tdslda_q1d_load_static(tdslda_ctx* c, int nprob, const double* kperp2, const double* hfield,
                                     const double* delta, double ecut, int64_t* nloaded) {
  return guard(c, [&] {
    require(c->q1d, TDSLDA_EINVAL, "static quasi-1D states need a quasi-1D context");
    require(kperp2 && hfield && delta && nprob > 0, TDSLDA_EINVAL, "bad problem list");
    const int64_t n = q1d_static(c->stream, c->lat.nz, c->lat.dz, nprob, kperp2, hfield, delta, ecut, nullptr,
                                 c->sb[0], c->esz, c->E, c->kperp2, c->cap);
    require(n > 0, TDSLDA_EINVAL, "no state below the cutoff");
    c->nst = n;
    hipLaunchKernelGGL(k_fill_real<double>, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, 1.0, c->mult);
    HIPCHK(hipGetLastError());
    set_weights(*c, n, nullptr);
    after_load(*c);
    if (nloaded) *nloaded = n;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_q1d_count_spin(const tdslda_lattice* lat, int nprob, const double* kperp2,
                                    const double* hfield_a, const double* hfield_b, const double* delta, double ecut,
                                    int32_t* counts, int64_t* total) {
  if (!lat || !kperp2 || !hfield_a || !hfield_b || !delta || nprob <= 0 || lat->mode != TDSLDA_MODE_Q1D)
    return TDSLDA_EINVAL;
  try {
    check_lattice(*lat);
    const int64_t t = q1d_static(nullptr, lat->nz, lat->dz, nprob, kperp2, hfield_a, delta, ecut, counts, nullptr,
                                 0, nullptr, nullptr, 0, hfield_b, true);
    if (total) *total = t;
    return TDSLDA_OK;
  } catch (const Fail& e) {
    std::fprintf(stderr, "tdslda_q1d_count_spin: %s\n", e.msg.c_str());
    return e.st;
  } catch (...) {
    return TDSLDA_EDEVICE;
  }
}

tdslda_status tdslda_q1d_load_static_spin(tdslda_ctx* c, int nprob, const double* kperp2, const double* hfield_a,
                                          const double* hfield_b, const double* delta, double ecut,
                                          int64_t* nloaded) {
  return guard(c, [&] {
    require(c->q1d, TDSLDA_EINVAL, "static quasi-1D states need a quasi-1D context");
    require(kperp2 && hfield_a && hfield_b && delta && nprob > 0, TDSLDA_EINVAL, "bad problem list");
    const int64_t n = q1d_static(c->stream, c->lat.nz, c->lat.dz, nprob, kperp2, hfield_a, delta, ecut, nullptr,
                                 c->sb[0], c->esz, c->E, c->kperp2, c->cap, hfield_b, true);
    require(n > 0, TDSLDA_EINVAL, "no state below the cutoff");
    c->nst = n;
    hipLaunchKernelGGL(k_fill_real<double>, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, 1.0, c->mult);
    HIPCHK(hipGetLastError());
    set_weights(*c, n, nullptr);
    after_load(*c);
    if (nloaded) *nloaded = n;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_energy(tdslda_ctx* c, double terms_out[9]) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states first");
    require(terms_out != nullptr, TDSLDA_EINVAL, "terms_out is NULL");
    energy(*c, terms_out);
  });
}

tdslda_status tdslda_check(tdslda_ctx* c, double out[3]) {
  tdslda_status extra = TDSLDA_OK;
  tdslda_status st = guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states first");
    double e[9];
    energy(*c, e);
    // norms of the stored state: 1/scale^2 must be 1 for a normalised state
    std::vector<double> sc(c->nst);
    norm_of(*c, c->phi);
    HIPCHK(hipMemcpyAsync(sc.data(), c->sscale[c->phi], 8 * c->nst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double worst = 0;
    bool finite = std::isfinite(e[5]) && std::isfinite(e[6]);
    for (double s : sc) {
      if (!std::isfinite(s) || s <= 0) {
        finite = false;
        continue;
      }
      worst = std::max(worst, std::fabs(1.0 / (s * s) - 1.0));
    }
    if (!c->have_ref) {
      c->have_ref = true;
      c->N0 = e[6];
      c->E0 = e[5] - c->fun.mu * e[6];
    }
    // conserved at fixed mu: Omega = E - mu N (Eq. E_tot); N itself is not
    // conserved when a pairing source Delta_ext acts
    const double dn = c->dext_on ? 0.0 : std::fabs(e[6] - c->N0) / std::fabs(c->N0);
    const double de = std::fabs(e[5] - c->fun.mu * e[6] - c->E0) / std::fabs(e[7]);
    if (out) {
      out[0] = dn;
      out[1] = de;
      out[2] = worst;
    }
    if (!finite) {
      c->err = "non-finite state norm or energy";
      extra = TDSLDA_EUNSTABLE;
    } else if ((c->run.tol_N > 0 && dn > c->run.tol_N) || (c->run.tol_E > 0 && de > c->run.tol_E)) {
      c->err = "conservation check failed: dN/N=" + std::to_string(dn) + " dE/E_FG=" + std::to_string(de);
      extra = TDSLDA_EUNSTABLE;
    }
  });
  return st != TDSLDA_OK ? st : extra;
}

tdslda_status tdslda_get_states(tdslda_ctx* c, double* uv) {
  return guard(c, [&] {
    require(c->loaded, TDSLDA_EORDER, "load states first");
    require(uv != nullptr, TDSLDA_EINVAL, "uv is NULL");
    const int64_t per = 2 * c->M;
    for (int64_t n0 = 0; n0 < c->nst; n0 += c->gchunk) {
      const int64_t k = std::min(c->gchunk, c->nst - n0);
      // scale into FP64 staging (per chunk, offset so state n0 lands at 0)
      PwDesc d;
      d.mode = PW_SCALE;
      d.X = (char*)c->sb[c->phi] + size_t(n0) * per * c->esz;
      d.scale = c->sscale[c->phi] + n0;
      d.out64 = c->gscratch;
      c->eng->pointwise(*c, d, k);
      HIPCHK(hipMemcpyAsync(uv + n0 * per * 2, c->gscratch, size_t(k) * per * 16, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_info(tdslda_ctx* c, int64_t* nstates, int64_t* steps, double* time) {
  return guard(c, [&] {
    if (nstates) *nstates = c->nst;
    if (steps) *steps = c->steps;
    if (time) *time = c->time;
  });
}

tdslda_status tdslda_save(tdslda_ctx* c, const char* path) {
  return guard(c, [&] {
    require(c->loaded && path, TDSLDA_EINVAL, "nothing to save or no path");
    FILE* f = std::fopen(path, "wb");
    require(f != nullptr, TDSLDA_EINVAL, std::string("cannot open ") + path);
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t per = 2 * c->M * c->esz;
    int64_t hdr[8] = {0x5444534c4442LL, c->nst, c->M, int64_t(c->esz), c->depth, c->steps, int64_t(c->started), int64_t(c->frozen)};
    std::vector<char> host(size_t(per) * std::min<int64_t>(c->nst, 256));
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(&c->time, 8, 1, f) == 1;
    int roles[6] = {c->phi, c->hist[0], c->hist[1], c->hist[2], c->hist[3], c->hist[4]};
    ok = ok && std::fwrite(roles, sizeof(roles), 1, f) == 1;
    auto dump = [&](const void* dev, size_t bytes) {
      std::vector<char> h(bytes);
      HIPCHK(hipMemcpy(h.data(), dev, bytes, hipMemcpyDeviceToHost));
      ok = ok && std::fwrite(h.data(), 1, bytes, f) == bytes;
    };
    for (int b = 0; b <= c->depth; ++b) {
      for (int64_t n0 = 0; n0 < c->nst; n0 += 256) {
        const int64_t k = std::min<int64_t>(256, c->nst - n0);
        HIPCHK(hipMemcpy(host.data(), (char*)c->sb[b] + n0 * per, size_t(k) * per, hipMemcpyDeviceToHost));
        ok = ok && std::fwrite(host.data(), 1, size_t(k) * per, f) == size_t(k) * per;
      }
      dump(c->sscale[b], 8 * c->nst);
    }
    dump(c->E, 8 * c->nst);
    dump(c->kperp2, 8 * c->nst);
    dump(c->vext, 8 * c->M);
    dump(c->lam, 8 * c->M);
    dump(c->U, 8 * c->M);
    dump(c->delta, 16 * c->M);
    dump(c->dext, 16 * c->M);
    // kinetic <H> partials left by the last producer kernel, so a resumed
    // run continues with exactly the arithmetic of an uninterrupted one
    int kin[6];
    for (int b = 0; b < 6; ++b) kin[b] = c->kin_ready[b] ? 1 : 0;
    ok = ok && std::fwrite(kin, sizeof(kin), 1, f) == 1;
    dump(c->h_part, 8 * size_t(c->nst) * c->h_stride);
    std::fclose(f);
    require(ok, TDSLDA_EINVAL, "short write");
  });
}

tdslda_status tdslda_load(tdslda_ctx* c, const char* path) {
  return guard(c, [&] {
    require(path != nullptr, TDSLDA_EINVAL, "no path");
    FILE* f = std::fopen(path, "rb");
    require(f != nullptr, TDSLDA_EINVAL, std::string("cannot open ") + path);
    int64_t hdr[8];
    double t;
    int roles[6];
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && std::fread(&t, 8, 1, f) == 1 &&
              std::fread(roles, sizeof(roles), 1, f) == 1;
    if (!ok || hdr[0] != 0x5444534c4442LL || hdr[2] != c->M || hdr[3] != int64_t(c->esz) || hdr[4] != c->depth ||
        hdr[1] > c->cap || hdr[1] <= 0) {
      std::fclose(f);
      throw Fail{TDSLDA_EINVAL, "checkpoint does not match this context"};
    }
    const int64_t n = hdr[1];
    const int64_t per = 2 * c->M * c->esz;
    std::vector<char> host(size_t(per) * std::min<int64_t>(n, 256));
    auto undump = [&](void* dev, size_t bytes) {
      std::vector<char> h(bytes);
      ok = ok && std::fread(h.data(), 1, bytes, f) == bytes;
      if (ok) HIPCHK(hipMemcpy(dev, h.data(), bytes, hipMemcpyHostToDevice));
    };
    for (int b = 0; b <= c->depth && ok; ++b) {
      for (int64_t n0 = 0; n0 < n && ok; n0 += 256) {
        const int64_t k = std::min<int64_t>(256, n - n0);
        ok = std::fread(host.data(), 1, size_t(k) * per, f) == size_t(k) * per;
        if (ok) HIPCHK(hipMemcpy((char*)c->sb[b] + n0 * per, host.data(), size_t(k) * per, hipMemcpyHostToDevice));
      }
      undump(c->sscale[b], 8 * n);
    }
    std::vector<double> E(n);
    ok = ok && std::fread(E.data(), 8, n, f) == size_t(n);
    undump(c->kperp2, 8 * n);
    undump(c->vext, 8 * c->M);
    undump(c->lam, 8 * c->M);
    undump(c->U, 8 * c->M);
    undump(c->delta, 16 * c->M);
    {
      std::vector<double> dx(2 * c->M);
      ok = ok && std::fread(dx.data(), 8, dx.size(), f) == dx.size();
      if (ok) HIPCHK(hipMemcpy(c->dext, dx.data(), 16 * c->M, hipMemcpyHostToDevice));
      c->dext_on = false;
      for (double v : dx) c->dext_on = c->dext_on || v != 0.0;
    }
    int kin[6] = {0, 0, 0, 0, 0, 0};
    ok = ok && std::fread(kin, sizeof(kin), 1, f) == 1;
    std::vector<double> hp(size_t(n) * c->h_stride);
    ok = ok && std::fread(hp.data(), 8, hp.size(), f) == hp.size();
    std::fclose(f);
    require(ok, TDSLDA_EINVAL, "short read");
    c->nst = n;
    set_weights(*c, n, E.data());
    c->phi = roles[0];
    for (int j = 0; j < 5; ++j) c->hist[j] = roles[j + 1];
    c->steps = hdr[5];
    c->started = hdr[6] != 0;
    c->time = t;
    c->loaded = true;
    c->have_ref = false;
    if (hdr[7]) {
      set_frozen_fields(*c);
      c->frozen = true;
    } else {
      c->frozen = false;
      c->eng->dens(*c, c->sb[c->phi], c->sscale[c->phi], c->nst);
      c->eng->reduce_pot(*c, true);
    }
    c->fields_valid = true;
    HIPCHK(hipMemcpyAsync(c->h_part, hp.data(), 8 * hp.size(), hipMemcpyHostToDevice, c->stream));
    for (int b = 0; b < 6; ++b) c->kin_ready[b] = kin[b] != 0;
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

tdslda_status tdslda_set_profiling(tdslda_ctx* c, int enable) {
  return guard(c, [&] {
    c->harvest();
    c->prof = enable != 0;
    for (int k = 0; k < KC_COUNT; ++k) {
      c->klaunch[k] = 0;
      c->kms[k] = 0;
    }
  });
}

tdslda_status tdslda_kernel_stats(tdslda_ctx* c, int k, int64_t* launches, double* total_ms) {
  if (!c) return TDSLDA_EINVAL;
  if (k < 0 || k >= KC_COUNT) return TDSLDA_EINVAL;
  return guard(c, [&] {
    c->harvest();
    if (launches) *launches = c->klaunch[k];
    if (total_ms) *total_ms = c->kms[k];
  });
}

}  // extern "C"
