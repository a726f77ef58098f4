// Quasi-2D kernel set (paper Sec. 3.1, quasi-2D item): every state is an
// N_x x N_y field phi(x, y) carrying its plane-wave momentum k_z^2 (the
// factor exp(i k_z z) / sqrt(L_z) is implicit); all |k_z| classes form one
// flat batch of states, so uneven per-class state counts need no special
// handling.  With A = 1 the problem of a class is the x-y BdG problem with
// the diagonal shifted by k_z^2 / 2 (mu -> mu - k_z^2 / 2).
//
// A state fits one workgroup: the 2D spectral Laplacian is done in LDS (y
// rows forward, x columns forward / multiply / back, y rows back, one thread
// per line; transforms of fft.h), so the evaluations that need <H>_n take it
// in the same pass (Parseval for the kinetic part while the columns are in
// k space, the potential part while the state is loaded) and fuse H phi,
// the shift and the integrator arithmetic as the full-3D lap2 does.
// Densities, potentials and pointwise passes are the transform-free kernels
// of the full-3D set applied to the M = N_x N_y sites of a state.
#include "ctx.h"

// largest sites-per-thread count for which the fused pass keeps its sites
// of phi in registers instead of re-reading them
#ifndef TDSLDA_Q2_STASH_MAXP
#define TDSLDA_Q2_STASH_MAXP 0
#endif

namespace tdslda {
namespace {

template <int NX, int NY>
struct Q2Cfg {
  static constexpr int M = NX * NY;
  static constexpr int NMAX = NX > NY ? NX : NY;
  // line phases: a lane pair per row / column (the lane-pair DFT of fft.h)
  static constexpr int TASKS = ((4 * NMAX + kWave - 1) / kWave) * kWave;  // line lanes (u and v)
  static constexpr int MW = ((M + kWave - 1) / kWave) * kWave;
  static constexpr int TB = TASKS > (MW < 256 ? MW : 256) ? TASKS : (MW < 256 ? MW : 256);
  static constexpr int P = (M + TB - 1) / TB;  // sites per thread
  static constexpr int PAD = NY + 2;           // LDS row pitch (bank spread of the lane pairs)
  static constexpr int LDS_ELEMS = 2 * NX * PAD;
  __device__ static int idx(int comp, int p) {
    const int x = p / NY, y = p - x * NY;
    return (comp * NX + x) * PAD + y;
  }
};

// <H>_n only (into h slot 0, slot 1 cleared): the shift of a prepared state
constexpr int Q2_EXPECT = 5;

// One workgroup per state n:
//   1. load s X_n (u, v) into LDS; with an own <H>_n the potential part
//      int [(hA + k_z^2/2)(|u|^2 - |v|^2) + 2 Re(u^* D v)] is summed here;
//   2. y rows forward (digit-reversed k_y along the row);
//   3. x columns forward; the kinetic part 1/2 (int |grad u|^2 - int |grad v|^2)
//      = +-1/2 dV / M sum_k k^2 |phi_k|^2 (Parseval); times -k^2 / M; back;
//   4. y rows back: LDS holds lap u, lap v (the full k^2 of Eq. D2);
//   5. H phi = (-1/2 lap u + a u + D v, D^* u + 1/2 lap v - a v) with
//      a = hA + k_z^2/2, f = -i (H - h) phi, then the mode's arithmetic
//      (see k_lap2): h = the own <H>_n in F / CORR / FULL, the given shift
//      in H / TAYLOR.
template <typename R, int NX, int NY, int MODE, int NP = 4, int NQ = 5>
__global__ __launch_bounds__((Q2Cfg<NX, NY>::TB)) void q2_lap(Lap2Args<R> A, const double* __restrict__ kz2,
                                                            double cx2, double cy2) {
  using CFG = Q2Cfg<NX, NY>;
  constexpr int TB = CFG::TB, P = CFG::P, M = CFG::M, PAD = CFG::PAD;
  constexpr bool OWN_H = MODE == L2_F || MODE == L2_CORR || MODE == L2_FULL || MODE == Q2_EXPECT;
  __shared__ cpx<R> lds[CFG::LDS_ELEMS];
  __shared__ double red[TB / kWave];
  const int tid = threadIdx.x;
  const int64_t n = blockIdx.x;
  constexpr int ES = sizeof(cpx<R>), RS = sizeof(R);
  const R s = A.scale ? R(A.scale[n]) : R(1);
  const double offd = 0.5 * kz2[n];
  const R off = R(offd);
  const int64_t so = n * 2 * M;
  const uint32_t SB = 2 * M * ES;
  const bi32x4 rX = make_rsrc(A.X + so, SB);
  const bi32x4 rA = make_rsrc(A.hA, M * RS);
  const bi32x4 rD = make_rsrc(A.hD, M * ES);
  const int vt = tid * ES;
  constexpr bool STASH = P <= TDSLDA_Q2_STASH_MAXP;
  cpx<R> xs[2][STASH ? P : 1];
  double hacc = 0.0;

#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int p = tid + i * TB;
    if (p < M) {
      const int o = i * TB * ES;
      const cpx<R> u = s * bload<R>(rX, vt, o), v = s * bload<R>(rX, vt, o + M * ES);
      lds[CFG::idx(0, p)] = u;
      lds[CFG::idx(1, p)] = v;
      if constexpr (STASH) {
        xs[0][i] = u;
        xs[1][i] = v;
      }
      if constexpr (OWN_H) {
        const double a = double(bload_real<R>(rA, tid * RS, i * TB * RS)) + offd;
        const cpx<R> D = bload<R>(rD, vt, o);
        const cpx<R> dv = D * v;  // u^* D v
        hacc += a * (norm2(u) - norm2(v)) +
                2.0 * (double(u.x) * double(dv.x) + double(u.y) * double(dv.y));
      }
    }
  }
  __syncthreads();
  // rows and columns are held by lane pairs: lane parity b owns the samples
  // 2j + b of its line; after the forward transforms, row (column) position
  // q holds the wave number pair_wavenum_at(q)
  const int lt = tid >> 1;
  const bool odd = tid & 1;
  constexpr int HX = NX / 2, HY = NY / 2;
  if (lt < 2 * NX) {  // y rows forward
    cpx<R>* base = lds + lt * PAD + (odd ? 1 : 0);
    cpx<R> a[HY];
#pragma unroll
    for (int j = 0; j < HY; ++j) a[j] = base[2 * j];
    fwd_pair<NY>(a, odd);
#pragma unroll
    for (int j = 0; j < HY; ++j) base[2 * j] = a[j];
  }
  __syncthreads();
  double kin = 0.0;
  if (lt < 2 * NY) {  // x columns: forward, (Parseval), times -k^2 / M, back
    const int comp = lt / NY, col = lt - comp * NY;
    cpx<R>* base = lds + (comp * NX + (odd ? 1 : 0)) * PAD + col;
    cpx<R> a[HX];
#pragma unroll
    for (int j = 0; j < HX; ++j) a[j] = base[2 * j * PAD];
    fwd_pair<NX>(a, odd);
    const int my = pair_wavenum_at<NY>(col);
    const double ey = cy2 * double(my * my);
    // k^2 = cx2 mx^2 + ey: the Parseval sum as two sums with integer
    // weights, the multiplier -k^2 / M formed per mode at its use
    const R fx = R(-cx2 / double(M)), fy = R(-ey / double(M));
    double sx = 0.0, s0 = 0.0;
    sfor<0, HX>::run([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const int mx = pair_wavenum<NX, j>(odd);
      if constexpr (OWN_H) {
        const double q = norm2(a[j]);
        s0 += q;
        sx += double(mx * mx) * q;
      }
      a[j] = (fx * R(mx * mx) + fy) * a[j];
    });
    if constexpr (OWN_H) kin = (comp == 0 ? 0.5 : -0.5) * (cx2 * sx + ey * s0) / double(M);
    inv_pair<NX>(a, odd);
#pragma unroll
    for (int j = 0; j < HX; ++j) base[2 * j * PAD] = a[j];
  }
  __syncthreads();
  if (lt < 2 * NX) {  // y rows back
    cpx<R>* base = lds + lt * PAD + (odd ? 1 : 0);
    cpx<R> a[HY];
#pragma unroll
    for (int j = 0; j < HY; ++j) a[j] = base[2 * j];
    inv_pair<NY>(a, odd);
#pragma unroll
    for (int j = 0; j < HY; ++j) base[2 * j] = a[j];
  }
  // the block sum synchronises before its first read of the shared slots,
  // which also orders the row pass before the pointwise reads below
  R h = A.hshift ? R(A.hshift[n]) : R(0);
  if constexpr (OWN_H) {
    const double ht = A.dV * block_sum<TB>(hacc + kin, red);
    if constexpr (MODE == Q2_EXPECT) {
      if (tid == 0) {
        A.h_part[n * A.h_stride] = ht;
        A.h_part[n * A.h_stride + 1] = 0.0;
      }
      return;
    }
    h = R(ht);
  } else {
    __syncthreads();
  }

  constexpr int HD = (NP > NQ - 1) ? NP : NQ - 1;  // history depth
  bi32x4 rO{}, rC{}, rAcc{}, rH[HD] = {};
  if constexpr (MODE != L2_CORR) rO = make_rsrc(A.out + so, SB);
  if constexpr (MODE == L2_TAYLOR) rAcc = make_rsrc(A.acc + so, SB);
  if constexpr (MODE == L2_CORR) rH[0] = make_rsrc(A.hist[0] + so, SB);
  if constexpr (MODE == L2_FULL) {
    rC = make_rsrc(A.cout + so, SB);
    sfor<1, HD>::run([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      rH[j] = make_rsrc(A.hist[j] + so, SB);
    });
  }
  double nacc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int p = tid + i * TB;
    if (p < M) {
      const int ou = i * TB * ES, ov = ou + M * ES;
      const cpx<R> lu = lds[CFG::idx(0, p)], lv = lds[CFG::idx(1, p)];
      const R fa = bload_real<R>(rA, tid * RS, i * TB * RS) + off;
      const cpx<R> D = bload<R>(rD, vt, ou);
      cpx<R> u, v;
      if constexpr (STASH) {
        u = xs[0][i];
        v = xs[1][i];
      } else {
        u = s * bload_nt<R>(rX, vt, ou);
        v = s * bload_nt<R>(rX, vt, ov);
      }
      const cpx<R> Hu = R(-0.5) * lu + fa * u + D * v;
      const cpx<R> Hv = conj(D) * u + R(0.5) * lv - fa * v;
      if constexpr (MODE == L2_H) {
        bstore_nt<R>(Hu, rO, vt, ou);
        bstore_nt<R>(Hv, rO, vt, ov);
      } else {
        const cpx<R> gu = Hu - h * u, gv = Hv - h * v;
        if constexpr (MODE == L2_TAYLOR) {
          const cpx<R> c{R(A.tay_re), R(A.tay_im)};
          const cpx<R> ou_ = c * gu, ov_ = c * gv;
          bstore_nt<R>(ou_, rO, vt, ou);
          bstore_nt<R>(ov_, rO, vt, ov);
          cpx<R> su, sv;
          if (A.init_acc) {
            su = u + ou_;
            sv = v + ov_;
          } else {
            su = bload_nt<R>(rAcc, vt, ou) + ou_;
            sv = bload_nt<R>(rAcc, vt, ov) + ov_;
          }
          bstore_nt<R>(su, rAcc, vt, ou);
          bstore_nt<R>(sv, rAcc, vt, ov);
          nacc += norm2(su) + norm2(sv);
        } else {
          const cpx<R> fu{gu.y, -gu.x}, fv{gv.y, -gv.x};  // -i g
          if constexpr (MODE == L2_F) {
            bstore_nt<R>(fu, rO, vt, ou);
            bstore_nt<R>(fv, rO, vt, ov);
          } else if constexpr (MODE == L2_CORR) {
            // phi_new = c + dt a_0 f(p), written over the input
            const R a0 = R(A.a[0]);
            const cpx<R> nu_ = bload_nt<R>(rH[0], vt, ou) + a0 * fu;
            const cpx<R> nv_ = bload_nt<R>(rH[0], vt, ov) + a0 * fv;
            bstore_nt<R>(nu_, rX, vt, ou);
            bstore_nt<R>(nv_, rX, vt, ov);
            nacc += norm2(nu_) + norm2(nv_);
          } else {  // L2_FULL: f_k, next predictor p (over the input), partial corrector c
            bstore_nt<R>(fu, rO, vt, ou);
            bstore_nt<R>(fv, rO, vt, ov);
            cpx<R> pu = u + R(A.b[0]) * fu, pv = v + R(A.b[0]) * fv;
            cpx<R> cu = u + R(A.a[1]) * fu, cv = v + R(A.a[1]) * fv;
            sfor<1, HD>::run([&](auto jc) {
              constexpr int j = decltype(jc)::value;
              const cpx<R> hu = bload_nt<R>(rH[j], vt, ou), hv = bload_nt<R>(rH[j], vt, ov);
              if constexpr (j < NP) {
                pu = pu + R(A.b[j]) * hu;
                pv = pv + R(A.b[j]) * hv;
              }
              if constexpr (j + 1 < NQ) {
                cu = cu + R(A.a[j + 1]) * hu;
                cv = cv + R(A.a[j + 1]) * hv;
              }
            });
            bstore_nt<R>(pu, rX, vt, ou);
            bstore_nt<R>(pv, rX, vt, ov);
            bstore_nt<R>(cu, rC, vt, ou);
            bstore_nt<R>(cv, rC, vt, ov);
            nacc += norm2(pu) + norm2(pv);
          }
        }
      }
    }
  }
  if (A.nrm_part) {
    const double t = block_sum<TB>(nacc, red);
    if (tid == 0) A.nrm_part[n * A.nrm_stride] = t;
  }
}

// energy path: the plane-wave part of tau, k_z^2 (w_v |v|^2 + w_u |u|^2),
// added to the per-state scratch the axis passes initialised, and j_z = 0
// (it cancels between +k_z and -k_z)
template <typename R>
__global__ __launch_bounds__(256) void q2_kz_tau(const cpx<R>* __restrict__ X, int64_t n0, int64_t M,
                                                 const double* __restrict__ scale, const double* __restrict__ wu,
                                                 const double* __restrict__ wv, const double* __restrict__ kz2,
                                                 double* __restrict__ tau_s, double* __restrict__ j_s) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t c = blockIdx.y, n = n0 + c;
  if (r >= M) return;
  const double s = scale[n];
  const cpx<R> u = X[n * 2 * M + r], v = X[n * 2 * M + M + r];
  tau_s[c * M + r] += kz2[n] * s * s * (wv[n] * norm2(v) + wu[n] * norm2(u));
  j_s[(c * 3 + 2) * M + r] = 0.0;
}

template <typename R, int NX, int NY>
struct EngineQ2D final : Engine {
  using CFG = Q2Cfg<NX, NY>;
  using PCFG = SlabCfg<1, NX, NY>;  // pointwise passes over a one-slab state
  static constexpr int M = NX * NY;
  static constexpr int DG = sizeof(R) == 8 ? 256 : 128;  // states per density group
  int ngx() const override { return 1; }
  int ncb() const override { return 1; }
  int group() const override { return DG; }
  size_t elem_size() const override { return sizeof(cpx<R>); }
  bool producer_kinetic() const override { return false; }
  bool self_shift() const override { return true; }
  int raw_h_slots() const override { return 0; }

  double cx2(const Ctx& c) const { double k = 2 * kPi / (NX * c.lat.dx); return k * k; }
  double cy2(const Ctx& c) const { double k = 2 * kPi / (NY * c.lat.dy); return k * k; }

  void dens(Ctx& c, const void* X, const double* scale, int64_t nst) override {
    const unsigned ng = cdiv(nst, DG);
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_dens_sum<R, DG>), dim3(cdiv(M, DS_TB * DS_P), ng), dim3(DS_TB), 0, c.stream,
                         (const cpx<R>*)X, nst, int64_t(M), c.wu, c.wv, scale, c.dens_part);
    });
    c.nsg_used = int(ng);
  }
  void reduce_pot(Ctx& c, bool update) override {
    FunParams fp{c.fun.functional, c.fun.B, c.fun.C, c.fun.inv_g_bdg, c.fun.mu, c.ainv, c.dext};
    c.launch(KC_REDUCE_POT, [&] {
      if (c.nsg_used >= 64 && M <= 4096)  // many state groups: one workgroup per site
        hipLaunchKernelGGL((k_reduce_pot_wide<R>), dim3(M), dim3(256), 0, c.stream, c.dens_part, c.nsg_used,
                           int64_t(M), fp, c.lam, c.vext, c.rho, c.nu, c.U, c.delta, (R*)c.hA, (cpx<R>*)c.hD,
                           int(update));
      else
        hipLaunchKernelGGL((k_reduce_pot<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, c.dens_part,
                           c.nsg_used, int64_t(M), fp, c.lam, c.vext, c.rho, c.nu, c.U, c.delta, (R*)c.hA,
                           (cpx<R>*)c.hD, int(update));
    });
  }
  Lap2Args<R> args(Ctx& c) const {
    Lap2Args<R> P{};
    P.hA = (const R*)c.hA;
    P.hD = (const cpx<R>*)c.hD;
    P.nrm_stride = c.nrm_stride;
    P.np = c.np;
    P.nq = c.nq;
    for (int i = 0; i < 5; ++i) {
      P.b[i] = c.bco[i];
      P.a[i] = c.aco[i];
    }
    P.h_part = c.h_part;
    P.h_stride = c.h_stride;
    P.dV = c.dV;
    return P;
  }
  // the start-up's shift: <H>_n of the scaled state into the h slots (no
  // intermediate buffer: every lap2 mode does its own transform)
  void lap1(Ctx& c, const void* X, const double* scale, bool hpart, int64_t nst) override {
    if (!hpart) return;
    Lap2Args<R> P = args(c);
    P.X = (const cpx<R>*)X;
    P.scale = scale;
    c.launch(KC_LAP1, [&] {
      hipLaunchKernelGGL((q2_lap<R, NX, NY, Q2_EXPECT>), dim3(nst), dim3(CFG::TB), 0, c.stream, P, c.kperp2,
                         cx2(c), cy2(c));
    });
  }
  void lap2(Ctx& c, const L2Desc& d, int64_t nst) override {
    Lap2Args<R> P = args(c);
    P.X = (const cpx<R>*)d.X;
    P.Xout = (cpx<R>*)d.Xout;
    P.scale = d.scale;
    P.hshift = d.hshift;
    P.out = (cpx<R>*)d.out;
    P.acc = (cpx<R>*)d.acc;
    for (int i = 0; i < 5; ++i) P.hist[i] = (const cpx<R>*)d.hist[i];
    P.cout = (cpx<R>*)d.cout;
    P.nrm_part = d.nrm_part;
    P.tay_re = d.tay_re;
    P.tay_im = d.tay_im;
    P.init_acc = d.init_acc;
    const dim3 grid(nst), block(CFG::TB);
    const double x2 = cx2(c), y2 = cy2(c);
    switch (d.mode) {
      case L2_H:
        c.launch(KC_LAP2_H, [&] { hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_H>), grid, block, 0, c.stream, P, c.kperp2, x2, y2); });
        break;
      case L2_F:
        c.launch(KC_LAP2_F, [&] { hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_F>), grid, block, 0, c.stream, P, c.kperp2, x2, y2); });
        break;
      case L2_CORR:
        c.launch(KC_LAP2_CORR, [&] { hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_CORR>), grid, block, 0, c.stream, P, c.kperp2, x2, y2); });
        break;
      case L2_FULL:
        c.launch(KC_LAP2_FULL, [&] {
          if (c.np == 3)
            hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_FULL, 3, 4>), grid, block, 0, c.stream, P, c.kperp2, x2, y2);
          else if (c.np == 5)
            hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_FULL, 5, 5>), grid, block, 0, c.stream, P, c.kperp2, x2, y2);
          else
            hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_FULL, 4, 5>), grid, block, 0, c.stream, P, c.kperp2, x2, y2);
        });
        break;
      default:
        c.launch(KC_LAP2_TAYLOR, [&] { hipLaunchKernelGGL((q2_lap<R, NX, NY, L2_TAYLOR>), grid, block, 0, c.stream, P, c.kperp2, x2, y2); });
    }
  }
  void pointwise(Ctx& c, const PwDesc& d, int64_t nst) override {
    PwArgs<R> A{};
    A.X = (cpx<R>*)d.X;
    A.scale = d.scale;
    for (int i = 0; i < 5; ++i) A.hist[i] = (const cpx<R>*)d.hist[i];
    A.cout = (cpx<R>*)d.cout;
    A.nrm_part = d.nrm_part;
    A.nrm_stride = c.nrm_stride;
    A.np = c.np;
    A.nq = c.nq;
    for (int i = 0; i < 5; ++i) {
      A.b[i] = c.bco[i];
      A.a[i] = c.aco[i];
    }
    A.out64 = (cpx<double>*)d.out64;
    A.nst = nst;
    const dim3 grid(1, state_rows(nst)), block(PCFG::TB);
    if (d.mode == PW_NORM)
      c.launch(KC_NORM, [&] { hipLaunchKernelGGL((k_pointwise<R, 1, NX, NY, PW_NORM>), grid, block, 0, c.stream, A); });
    else if (d.mode == PW_PRED)
      c.launch(KC_PRED, [&] {
        if (c.np == 3)
          hipLaunchKernelGGL((k_pointwise<R, 1, NX, NY, PW_PRED, 3, 4>), grid, block, 0, c.stream, A);
        else if (c.np == 5)
          hipLaunchKernelGGL((k_pointwise<R, 1, NX, NY, PW_PRED, 5, 5>), grid, block, 0, c.stream, A);
        else
          hipLaunchKernelGGL((k_pointwise<R, 1, NX, NY, PW_PRED, 4, 5>), grid, block, 0, c.stream, A);
      });
    else
      c.launch(KC_SETUP, [&] { hipLaunchKernelGGL((k_pointwise<R, 1, NX, NY, PW_SCALE>), grid, block, 0, c.stream, A); });
  }
  void friction(Ctx& c, const void* X, const double* scale, int64_t nst) override {
    (void)c, (void)X, (void)scale, (void)nst;
    throw Fail{TDSLDA_EINVAL, "quantum friction is not built for the quasi-2D kernel set"};
  }
  // tau and j: x and y line passes (D1 with the Nyquist mode zeroed, the
  // Nyquist amplitude at full weight), then the k_z^2 term of tau
  void grad(Ctx& c, const void* X, const double* scale, int64_t n0, int64_t nchunk) override {
    constexpr int TBG = 64;
    double* ts = c.gscratch;
    double* js = c.gscratch + nchunk * M;
    const double px = kPi / c.lat.dx, py = kPi / c.lat.dy;
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((k_grad_axis<R, NX, 0, TBG>), dim3(cdiv(M / NX, TBG), nchunk), dim3(TBG), 0, c.stream,
                         (const cpx<R>*)X, n0, nchunk, int64_t(M), int64_t(NY), int64_t(NY), scale, c.wu, c.wv,
                         2 * kPi / (NX * c.lat.dx), px * px, ts, js);
    });
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((k_grad_axis<R, NY, 1, TBG>), dim3(cdiv(M / NY, TBG), nchunk), dim3(TBG), 0, c.stream,
                         (const cpx<R>*)X, n0, nchunk, int64_t(M), int64_t(1), int64_t(1), scale, c.wu, c.wv,
                         2 * kPi / (NY * c.lat.dy), py * py, ts, js);
    });
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((q2_kz_tau<R>), dim3(cdiv(M, 256), nchunk), dim3(256), 0, c.stream, (const cpx<R>*)X, n0,
                         int64_t(M), scale, c.wu, c.wv, c.kperp2, ts, js);
    });
  }
};

template <typename R>
std::unique_ptr<Engine> make_q2d(int nx, int ny) {
  if (nx == 8 && ny == 8) return std::unique_ptr<Engine>(new EngineQ2D<R, 8, 8>());
  if (nx == 12 && ny == 12) return std::unique_ptr<Engine>(new EngineQ2D<R, 12, 12>());
  if (nx == 16 && ny == 16) return std::unique_ptr<Engine>(new EngineQ2D<R, 16, 16>());
  if (nx == 24 && ny == 16) return std::unique_ptr<Engine>(new EngineQ2D<R, 24, 16>());
  if (nx == 32 && ny == 32) return std::unique_ptr<Engine>(new EngineQ2D<R, 32, 32>());
  if (nx == 48 && ny == 48) return std::unique_ptr<Engine>(new EngineQ2D<R, 48, 48>());
  if (nx == 64 && ny == 64) return std::unique_ptr<Engine>(new EngineQ2D<R, 64, 64>());
  return nullptr;
}

}  // namespace

std::unique_ptr<Engine> make_q2d_f64(int nx, int ny) { return make_q2d<double>(nx, ny); }
std::unique_ptr<Engine> make_q2d_f32(int nx, int ny) { return make_q2d<float>(nx, ny); }

}  // namespace tdslda
