// Device kernels of the general functional (A != 1; Sec. 2.3, Eq. h_sigma)
// on the full 3D lattice.  The single-particle Hamiltonian carries an
// inverse effective mass alpha(r) and a current potential A(r):
//   h = -1/2 div(alpha grad) + hfield - (i/2) {A, grad},
// the kinetic part in the symmetrised form of Eq. kinop-alpha,
//   K x = -1/4 [lap(alpha x) + alpha lap x - x lap alpha],
// the current part as the anticommutator of the matrix forms of Eqs. Ad_dx
// and d_dxA, C x = -(i/2) sum_d [A_d D1_d x + D1_d(A_d x)] (D1 with the
// Nyquist bin zeroed, D2 with the full k^2).  Rows: u -> K u + C u +
// hfield u + Delta v;  v -> -K v + C v - hfield v + Delta^* u.
//
// Every derivative is taken along one axis at a time by a line pass (one
// thread owns one line of one state and transforms it in registers):
//   k_jline  - the current j_d of a group of states (field builds),
//   k_opline - the d-part of K and C of every state into T; the last axis
//              adds the local terms (T = H phi) and the partials of <H>_n,
// and k_pw_gen does the integrator arithmetic from T = H phi pointwise.
#pragma once

#include "kernels3d.h"

namespace tdslda {

// lines along AXIS of an NX x NY x NZ lattice: line l enumerates (outer,
// inner) with the axis between; site(l, k) = site0(l) + k STRIDE
template <int NX, int NY, int NZ, int AXIS>
struct LineGeo {
  static constexpr int NL = AXIS == 0 ? NX : (AXIS == 1 ? NY : NZ);
  static constexpr int STRIDE = AXIS == 0 ? NY * NZ : (AXIS == 1 ? NZ : 1);
  static constexpr int NLINES = NX * NY * NZ / NL;
  __device__ static int site0(int l) {
    const int outer = l / STRIDE, in = l - outer * STRIDE;
    return outer * STRIDE * NL + in;
  }
};

// j_AXIS group partials over DG states of the normalised states:
//   jpart[g][AXIS][site] = sum_n f_v Im(v (D1 v)^*) - f_u Im(u (D1 u)^*)
// (a component of zero weight is skipped: f_u = 0 for E > 0 at T = 0).
// A lane pair per line (lane parity b: samples 2j + b).
//   grid = (ceil(NLINES / (TBG / 2)), number of groups), block = TBG
template <typename R, int NX, int NY, int NZ, int AXIS, int TBG, int DG>
__global__ __launch_bounds__(TBG) void k_jline(const cpx<R>* __restrict__ X, int64_t nstates,
                                               const double* __restrict__ scale, const double* __restrict__ wu,
                                               const double* __restrict__ wv, double kscale,
                                               double* __restrict__ jpart) {
  using LG = LineGeo<NX, NY, NZ, AXIS>;
  constexpr int NL = LG::NL, ST = LG::STRIDE, HL = NL / 2;
  constexpr int64_t M = int64_t(NX) * NY * NZ;
  constexpr int ES = sizeof(cpx<R>);
  const int l = blockIdx.x * (TBG / 2) + threadIdx.x / 2;
  const bool odd = threadIdx.x & 1;
  if (l >= LG::NLINES) return;  // both lanes of a pair; no barriers below
  const int s0 = LG::site0(l) + (odd ? ST : 0);
  const int64_t nbeg = int64_t(blockIdx.y) * DG;
  const int nloc = int(nstates - nbeg < DG ? nstates - nbeg : DG);
  double acc[HL];
#pragma unroll
  for (int j = 0; j < HL; ++j) acc[j] = 0.0;
  for (int ls = 0; ls < nloc; ++ls) {
    const int64_t n = nbeg + ls;
    const R s = R(scale[n]);
    const double fu = wu[n], fv = wv[n];
    const bi32x4 rX = make_rsrc(X + n * 2 * M, uint32_t(2 * M * ES));
#pragma unroll 1
    for (int comp = 0; comp < 2; ++comp) {
      const double w = comp ? fv : -fu;
      if (w == 0.0) continue;  // uniform over the block
      cpx<R> d[HL], ny;
#pragma unroll
      for (int j = 0; j < HL; ++j) d[j] = s * bload<R>(rX, s0 * ES, int(comp * M + 2 * j * ST) * ES);
      first_derivative_pair<NL>(d, R(kscale), odd, ny);
#pragma unroll
      for (int j = 0; j < HL; ++j) {
        const cpx<R> f = s * bload<R>(rX, s0 * ES, int(comp * M + 2 * j * ST) * ES);  // re-read (cached)
        acc[j] += w * (double(f.y) * double(d[j].x) - double(f.x) * double(d[j].y));  // Im(f (D1 f)^*)
      }
    }
  }
  double* out = jpart + (int64_t(blockIdx.y) * 3 + AXIS) * M + s0;
#pragma unroll
  for (int j = 0; j < HL; ++j) out[2 * j * ST] = acc[j];
}

// Spin-imbalanced ASLDA (Sec. 2.4, ASLDA item; Eqs. na3D-jb3D), both
// branches evolved: the AXIS part of tau_s and j_s of a group of DG states,
// per line, into the [group][12][M] layout (0 rho_a, 1 rho_b, 2 Re nu,
// 3 Im nu from the transform-free pass; 4 tau_a, 5 tau_b; 6..8 j_a,
// 9..11 j_b by axis):
//   tau_a += sum f_u (|D1 u|^2 + (pi/d)^2 |c_u|^2),  tau_b with v, f_v
//   (AXIS 0 writes, the other axes add), j_a,AXIS = -sum f_u Im(u (D1 u)^*),
//   j_b,AXIS = sum f_v Im(v (D1 v)^*); D1 with the Nyquist bin zeroed, c the
//   Nyquist amplitude.  A lane pair per line (lane parity b: samples 2j + b).
//   grid = (ceil(NLINES / (TBG / 2)), number of groups), block = TBG
template <typename R, int NX, int NY, int NZ, int AXIS, int TBG, int DG>
__global__ __launch_bounds__(TBG) void k_taujline(const cpx<R>* __restrict__ X, int64_t nstates,
                                                  const double* __restrict__ scale, const double* __restrict__ wu,
                                                  const double* __restrict__ wv, double kscale, double nyq2,
                                                  double* __restrict__ part) {
  using LG = LineGeo<NX, NY, NZ, AXIS>;
  constexpr int NL = LG::NL, ST = LG::STRIDE, HL = NL / 2;
  constexpr int64_t M = int64_t(NX) * NY * NZ;
  constexpr int ES = sizeof(cpx<R>);
  const int l = blockIdx.x * (TBG / 2) + threadIdx.x / 2;
  const bool odd = threadIdx.x & 1;
  if (l >= LG::NLINES) return;  // both lanes of a pair; no barriers below
  const int s0 = LG::site0(l) + (odd ? ST : 0);
  const int64_t nbeg = int64_t(blockIdx.y) * DG;
  const int nloc = int(nstates - nbeg < DG ? nstates - nbeg : DG);
  double* gp = part + int64_t(blockIdx.y) * 12 * M + s0;
#pragma unroll 1
  for (int comp = 0; comp < 2; ++comp) {
    const double sgn = comp ? 1.0 : -1.0;
    double at[HL], aj[HL];
#pragma unroll
    for (int j = 0; j < HL; ++j) at[j] = aj[j] = 0.0;
    for (int ls = 0; ls < nloc; ++ls) {
      const int64_t n = nbeg + ls;
      const double w = comp ? wv[n] : wu[n];
      if (w == 0.0) continue;  // uniform over the block
      const R s = R(scale[n]);
      const bi32x4 rX = make_rsrc(X + n * 2 * M, uint32_t(2 * M * ES));
      cpx<R> d[HL], ny;
#pragma unroll
      for (int j = 0; j < HL; ++j) d[j] = s * bload<R>(rX, s0 * ES, int(comp * M + 2 * j * ST) * ES);
      first_derivative_pair<NL>(d, R(kscale), odd, ny);
      const double cn = nyq2 * norm2(ny);
#pragma unroll
      for (int j = 0; j < HL; ++j) {
        const cpx<R> f = s * bload<R>(rX, s0 * ES, int(comp * M + 2 * j * ST) * ES);  // re-read (cached)
        at[j] += w * (norm2(d[j]) + cn);
        aj[j] += sgn * w * (double(f.y) * double(d[j].x) - double(f.x) * double(d[j].y));  // Im(f (D1 f)^*)
      }
    }
    double* ot = gp + (4 + comp) * M;
    double* oj = gp + (6 + 3 * comp + AXIS) * M;
#pragma unroll
    for (int j = 0; j < HL; ++j) {
      if constexpr (AXIS == 0)
        ot[2 * j * ST] = at[j];
      else
        ot[2 * j * ST] += at[j];
      oj[2 * j * ST] = aj[j];
    }
  }
}

// ASLDA parameters (Sec. 2.4): A(p), A'(p), B(p), B'(p)
__device__ __forceinline__ double as3_A(double p) {
  const double p2 = p * p;
  return 1.094 + 0.156 * p * (1.0 - 2.0 * p2 / 3.0 + p2 * p2 / 5.0) - 0.532 * p2 * (1.0 - p2 + p2 * p2 / 3.0);
}
__device__ __forceinline__ double as3_dA(double p) {
  const double p2 = p * p;
  return 0.156 * (1.0 - 2.0 * p2 + p2 * p2) - 0.532 * (2.0 * p - 4.0 * p2 * p + 2.0 * p2 * p2 * p);
}
__device__ __forceinline__ double as3_B(double p) {
  const double hp = 0.5 * (1.0 + p), hm = 0.5 * (1.0 - p);
  return 1.5874010519681994 * (0.357 + 0.642 * p * p - as3_A(p) * pow(hp, 5.0 / 3.0) - as3_A(-p) * pow(hm, 5.0 / 3.0));
}
__device__ __forceinline__ double as3_dB(double p) {
  const double hp = 0.5 * (1.0 + p), hm = 0.5 * (1.0 - p);
  return 1.5874010519681994 *
         (1.284 * p - as3_dA(p) * pow(hp, 5.0 / 3.0) - as3_A(p) * (5.0 / 6.0) * pow(hp, 2.0 / 3.0) +
          as3_dA(-p) * pow(hm, 5.0 / 3.0) + as3_A(-p) * (5.0 / 6.0) * pow(hm, 2.0 / 3.0));
}

// one thread per site: the twelve group partials summed in a fixed order,
// then the ASLDA potentials (functional derivatives of the SLDA-type energy
// density with A_a = A(p), A_b = A(-p), B(p); see the quasi-1D kernel set):
//   V_s = dp/drho_s [1/2 (A'(p) K_a - A'(-p) K_b) + 3/5 B'(p) rho_+ eF]
//         + (A_s - 1) |j_s|^2 / (2 rho_s^2) + B eF - |Delta|^2 / (3 C rho_+^(2/3)),
//   A_s = (1 - A_s) j_s / rho_s (three components), Delta = -g_eff nu,
// spin-resolved arrays [spin][M] (j: [spin][3][M]); alpha_s into aout.
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_aslda3d(
    const double* __restrict__ part, int ngroups, int64_t M, FunParams fp, double mu_b,
    const double* __restrict__ lam, const double* __restrict__ vext, double* __restrict__ rho,
    double* __restrict__ tau, double* __restrict__ nu, double* __restrict__ jc, double* __restrict__ U,
    double* __restrict__ delta, R* __restrict__ hA, cpx<R>* __restrict__ hD, R* __restrict__ hAx,
    R* __restrict__ hAy, R* __restrict__ hAz, double* __restrict__ aout, int update_fields) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const double* p = part + int64_t(g) * 12 * M + r;
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] += p[c * M];
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] *= fp.ainv;
  rho[r] = v[0];
  rho[M + r] = v[1];
  nu[2 * r] = v[2];
  nu[2 * r + 1] = v[3];
  tau[r] = v[4];
  tau[M + r] = v[5];
#pragma unroll
  for (int c = 0; c < 6; ++c) jc[c * M + r] = v[6 + c];
  if (!update_fields) return;
  const double ra = fmax(v[0], 0.5e-14), rb = fmax(v[1], 0.5e-14), rp = ra + rb;
  const double p = (ra - rb) / rp;
  const double Aa = as3_A(p), Ab = as3_A(-p), B = as3_B(p);
  const double gg = 1.0 / (cbrt(rp) / fp.C - lam[r]);
  const double dr = -gg * v[2], di = -gg * v[3];
  const double ef = 0.5 * pow(3.0 * kPi * kPi * rp, 2.0 / 3.0);
  const double c23 = cbrt(rp);
  const double jsa = v[6] * v[6] + v[7] * v[7] + v[8] * v[8], jsb = v[9] * v[9] + v[10] * v[10] + v[11] * v[11];
  const double Ka = v[4] - jsa / ra, Kb = v[5] - jsb / rb;
  const double common = 0.5 * (as3_dA(p) * Ka - as3_dA(-p) * Kb) + 0.6 * as3_dB(p) * rp * ef;
  const double base = B * ef - (dr * dr + di * di) / (3.0 * fp.C * c23 * c23);
  const double Va = 2.0 * rb / (rp * rp) * common + (Aa - 1.0) * jsa / (2.0 * ra * ra) + base;
  const double Vb = -2.0 * ra / (rp * rp) * common + (Ab - 1.0) * jsb / (2.0 * rb * rb) + base;
  U[r] = Va;
  U[M + r] = Vb;
  delta[2 * r] = dr;
  delta[2 * r + 1] = di;
  hA[r] = R(Va + vext[r] - fp.mu);
  hA[M + r] = R(Vb + vext[r] - mu_b);
  hD[r] = cpx<R>{R(dr + fp.dext[2 * r]), R(di + fp.dext[2 * r + 1])};
  const double ca = (1.0 - Aa) / ra, cb = (1.0 - Ab) / rb;
  hAx[r] = R(ca * v[6]);
  hAy[r] = R(ca * v[7]);
  hAz[r] = R(ca * v[8]);
  hAx[M + r] = R(cb * v[9]);
  hAy[M + r] = R(cb * v[10]);
  hAz[M + r] = R(cb * v[11]);
  aout[r] = Aa;
  aout[M + r] = Ab;
}

// A compiler-only memory fence (no instruction): the phases of a line pass
// re-read phi and the fields instead of keeping them in registers across
// the transforms (the loads would otherwise be merged or hoisted, which
// costs more registers than the re-reads cost bandwidth)
__device__ __forceinline__ void phase_fence() { __asm__ volatile("" ::: "memory"); }

// -(i/2) c
template <typename R>
__device__ __forceinline__ cpx<R> minus_half_i(cpx<R> c) {
  return cpx<R>{R(0.5) * c.y, R(-0.5) * c.x};
}

// The AXIS part of K and C of every state, row-signed, into T (the FIRST
// pass writes, the others add); LAST also adds the local terms,
//   u: + (1/4 lap alpha + hfield) u + Delta v,  v: - (1/4 lap alpha + hfield) v + Delta^* u,
// so that the destination (out when given, else T) holds H phi, and when
// h_part is given writes the block's partial of <H>_n = Re int phi^* H phi
// dV into h slot h_off + blockIdx.x; block 0 clears the slots [0, h_off)
// and [h_off + gridDim.x, h_off + n_slots).  phi = scale x X (scale NULL = 1).
// Each line is held by a lane pair (the lane-pair DFT of fft.h: lane parity
// b owns the samples 2j + b), which halves the registers of a line.
//   grid = (ceil(NLINES / (TBG / 2)), nstates), block = TBG
template <typename R, int NX, int NY, int NZ, int AXIS, int TBG, bool FIRST, bool LAST>
__global__ __launch_bounds__(TBG) void k_opline(const cpx<R>* __restrict__ X, const double* __restrict__ scale,
                                                cpx<R>* __restrict__ T, cpx<R>* __restrict__ out,
                                                const R* __restrict__ hAl, const R* __restrict__ hLa,
                                                const R* __restrict__ hAd, const R* __restrict__ hA,
                                                const cpx<R>* __restrict__ hD, double* __restrict__ h_part,
                                                int h_stride, int h_off, int n_slots, double kscale, double dV,
                                                int64_t fcs) {
  using LG = LineGeo<NX, NY, NZ, AXIS>;
  constexpr int NL = LG::NL, ST = LG::STRIDE, HL = NL / 2;
  static_assert(NL % 2 == 0 && TBG % kWave == 0, "lane pairs");
  constexpr int64_t M = int64_t(NX) * NY * NZ;
  constexpr int ES = sizeof(cpx<R>), RS = sizeof(R);
  __shared__ double red[TBG / kWave];
  // the running sum of the line's terms, sample j of this lane at [j][lane]:
  // one half-line array stays in registers
  __shared__ cpx<R> acc[HL][TBG];
  const int tx = threadIdx.x;
  const int l = blockIdx.x * (TBG / 2) + tx / 2;
  const bool odd = tx & 1;
  const bool act = l < LG::NLINES;  // the same for both lanes of a pair
  const int s0 = (act ? LG::site0(l) : 0) + (odd ? ST : 0);  // this lane's first sample
  const int64_t n = blockIdx.y;
  const R s = scale ? R(scale[n]) : R(1);
  const uint32_t SB = uint32_t(2 * M * ES);
  const bi32x4 rX = make_rsrc(X + n * 2 * M, SB);
  const bi32x4 rT = make_rsrc(T + n * 2 * M, SB);
  cpx<R>* dst = (LAST && out) ? out : T;
  const bi32x4 rO = make_rsrc(dst + n * 2 * M, SB);
  const int vo = s0 * ES, va = s0 * RS;
  const R kk = R(kscale), inv_n = R(1.0 / NL);
  double hloc = 0.0;
  // spectral factors at position p: -k^2 / N (D2, the Nyquist bin kept) and
  // i k / N (D1, the Nyquist bin zeroed)
  auto d2 = [&](cpx<R>(&t)[HL]) {
    sfor<0, HL>::run([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      const R km = kk * R(pair_wavenum<NL, p>(odd));
      t[p] = (-km * km * inv_n) * t[p];
    });
  };
  auto d1 = [&](cpx<R>(&t)[HL]) {
    sfor<0, HL>::run([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      const int m = pair_wavenum<NL, p>(odd);
      const R km = (m == -HL) ? R(0) : kk * R(m);
      t[p] = (km * inv_n) * mul_i(t[p]);
    });
  };
  if (act) {
#pragma unroll 1
    for (int comp = 0; comp < 2; ++comp) {
      const R sg = comp ? R(-1) : R(1);
      const int cb = int(comp * M);
      // the fields of this row's spin (fcs = M: [spin][M] arrays; 0: one set)
      const int64_t fo = comp * fcs;
      const bi32x4 rAl = make_rsrc(hAl + fo, uint32_t(M * RS)), rAd = make_rsrc(hAd + fo, uint32_t(M * RS));
      cpx<R> t[HL];
      phase_fence();
      // D2(alpha x) and D1(A_d x) share one inverse transform: the first
      // spectrum waits in the running-sum slots (each lane's own positions)
#pragma unroll
      for (int j = 0; j < HL; ++j)
        t[j] = bload_real<R>(rAl, va, 2 * j * ST * RS) * (s * bload<R>(rX, vo, (cb + 2 * j * ST) * ES));
      fwd_pair<NL>(t, odd);
      d2(t);
#pragma unroll
      for (int j = 0; j < HL; ++j) acc[j][tx] = (sg * R(-0.25)) * t[j];
      phase_fence();
#pragma unroll
      for (int j = 0; j < HL; ++j)
        t[j] = bload_real<R>(rAd, va, 2 * j * ST * RS) * (s * bload<R>(rX, vo, (cb + 2 * j * ST) * ES));
      fwd_pair<NL>(t, odd);
      d1(t);
#pragma unroll
      for (int j = 0; j < HL; ++j) t[j] = acc[j][tx] + minus_half_i(t[j]);
      inv_pair<NL>(t, odd);
#pragma unroll
      for (int j = 0; j < HL; ++j) acc[j][tx] = t[j];
      phase_fence();
      // alpha D2 x
#pragma unroll
      for (int j = 0; j < HL; ++j) t[j] = s * bload<R>(rX, vo, (cb + 2 * j * ST) * ES);
      fwd_pair<NL>(t, odd);
      d2(t);
      inv_pair<NL>(t, odd);
#pragma unroll
      for (int j = 0; j < HL; ++j)
        acc[j][tx] = acc[j][tx] + (sg * R(-0.25) * bload_real<R>(rAl, va, 2 * j * ST * RS)) * t[j];
      phase_fence();
      // A_d D1 x
#pragma unroll
      for (int j = 0; j < HL; ++j) t[j] = s * bload<R>(rX, vo, (cb + 2 * j * ST) * ES);
      fwd_pair<NL>(t, odd);
      d1(t);
      inv_pair<NL>(t, odd);
      phase_fence();
#pragma unroll
      for (int j = 0; j < HL; ++j) {
        cpx<R> r = acc[j][tx] + minus_half_i(bload_real<R>(rAd, va, 2 * j * ST * RS) * t[j]);
        const int o = (cb + 2 * j * ST) * ES;
        if constexpr (!FIRST) r = r + bload<R>(rT, vo, o);
        if constexpr (LAST) {
          // per-site fields through buffer resources: the sample's row as a
          // scalar offset, no per-sample address registers
          const bi32x4 rD = make_rsrc(hD, uint32_t(M * ES));
          const bi32x4 rLa = make_rsrc(hLa, uint32_t((M + fcs) * RS)), rHA = make_rsrc(hA, uint32_t((M + fcs) * RS));
          const int fs = int(fo + 2 * j * ST) * RS;
          const cpx<R> x = s * bload<R>(rX, vo, o);
          const cpx<R> y = s * bload<R>(rX, vo, (int((1 - comp) * M) + 2 * j * ST) * ES);
          const cpx<R> D = bload<R>(rD, vo, 2 * j * ST * ES);
          const cpx<R> Dc = comp ? conj(D) : D;
          r = r + (sg * (R(0.25) * bload_real<R>(rLa, va, fs) + bload_real<R>(rHA, va, fs))) * x + Dc * y;
          hloc += double(x.x) * double(r.x) + double(x.y) * double(r.y);
        }
        bstore<R>(r, rO, vo, o);
      }
    }
  }
  if constexpr (LAST) {
    if (h_part) {
      double v = wave_sum(hloc);
      if (tx % kWave == 0) red[tx / kWave] = v;
      __syncthreads();
      if (tx == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < TBG / kWave; ++w) t += red[w];
        double* hp = h_part + n * h_stride;
        hp[h_off + blockIdx.x] = t * dV;
        if (blockIdx.x == 0) {
          for (int i = 0; i < h_off; ++i) hp[i] = 0.0;
          for (int i = int(gridDim.x); i < n_slots; ++i) hp[h_off + i] = 0.0;
        }
      }
    }
  }
}

// The integrator arithmetic from T = H phi (built by k_opline), pointwise
// over the slab tiling of k_pointwise; phi = scale x X, h = hshift[n]:
//   H: out = T;  F: out = -i (T - h phi);  TAYLOR: out = c (T - h phi), acc
//   += out;  CORR: phi_new = c + dt a_0 f;  FULL: f_k, next predictor p
//   (over the input), partial corrector c; norm partials of the written
//   state per slab group (as k_lap2).
//   grid = (NGX, nstates), block = TB
template <typename R, int NX, int NY, int NZ, int MODE, int NP = 4, int NQ = 5>
__global__ __launch_bounds__((SlabCfg<NX, NY, NZ>::TB)) void k_pw_gen(Lap2Args<R> A) {
  using CFG = SlabCfg<NX, NY, NZ>;
  constexpr int TB = CFG::TB, P = CFG::P, SS = CFG::SS;
  constexpr int M = NX * NY * NZ;
  constexpr int HD = (NP > NQ - 1) ? NP : NQ - 1;
  __shared__ double red[TB / kWave];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t n = blockIdx.y;
  constexpr int ES = sizeof(cpx<R>);
  const int64_t so = n * 2 * M;
  const uint32_t SB = 2 * M * ES;
  const R s = A.scale ? R(A.scale[n]) : R(1);
  const R h = A.hshift ? R(A.hshift[n]) : R(0);
  const bi32x4 rX = make_rsrc(A.X + so, SB);
  const bi32x4 rT = make_rsrc(A.T + so, SB);
  bi32x4 rO{}, rXo{}, rC{}, rAcc{}, rH[HD] = {};
  if constexpr (MODE != L2_CORR) rO = make_rsrc(A.out + so, SB);
  if constexpr (MODE == L2_CORR || MODE == L2_FULL) rXo = make_rsrc(A.Xout + so, SB);
  if constexpr (MODE == L2_TAYLOR) rAcc = make_rsrc(A.acc + so, SB);
  if constexpr (MODE == L2_CORR) rH[0] = make_rsrc(A.hist[0] + so, SB);
  if constexpr (MODE == L2_FULL) {
    rC = make_rsrc(A.cout + so, SB);
    sfor<1, HD>::run([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      rH[j] = make_rsrc(A.hist[j] + so, SB);
    });
  }
  const int vt = tid * ES;
  double nacc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int p = tid + i * TB;
    if (p < SS) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int o = int(int64_t(g) * SS + i * TB + c * M) * ES;
        const cpx<R> hx = bload<R>(rT, vt, o);
        if constexpr (MODE == L2_H) {
          bstore<R>(hx, rO, vt, o);
        } else {
          const cpx<R> x = s * bload<R>(rX, vt, o);
          const cpx<R> gg = hx - h * x;
          if constexpr (MODE == L2_TAYLOR) {
            const cpx<R> cf{R(A.tay_re), R(A.tay_im)};
            const cpx<R> ov = cf * gg;
            const cpx<R> sm = A.init_acc ? x + ov : bload<R>(rAcc, vt, o) + ov;
            bstore<R>(ov, rO, vt, o);
            bstore<R>(sm, rAcc, vt, o);
            nacc += norm2(sm);
          } else {
            const cpx<R> f{gg.y, -gg.x};  // -i g
            if constexpr (MODE == L2_F) {
              bstore<R>(f, rO, vt, o);
            } else if constexpr (MODE == L2_CORR) {
              const cpx<R> nw = bload<R>(rH[0], vt, o) + R(A.a[0]) * f;
              bstore<R>(nw, rXo, vt, o);
              nacc += norm2(nw);
            } else {  // L2_FULL
              cpx<R> pp = x + R(A.b[0]) * f, cc = x + R(A.a[1]) * f;
              sfor<1, HD>::run([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const cpx<R> hj = bload<R>(rH[j], vt, o);
                if constexpr (j < NP) pp = pp + R(A.b[j]) * hj;
                if constexpr (j + 1 < NQ) cc = cc + R(A.a[j + 1]) * hj;
              });
              bstore<R>(f, rO, vt, o);
              bstore<R>(pp, rXo, vt, o);
              bstore<R>(cc, rC, vt, o);
              nacc += norm2(pp);
            }
          }
        }
      }
    }
  }
  if (A.nrm_part && MODE != L2_H && MODE != L2_F) {
    const double t = block_sum<TB>(nacc, red);
    if (tid == 0) A.nrm_part[n * A.nrm_stride + g] = t;
  }
}

// Sums of the density and the current group partials (fixed order, one thread
// per site) and the potentials of the SLDA functional at A != 1
// (spin-symmetric, per spin): Delta = -g_eff nu, U = B eF - |Delta|^2 /
// (3 C rho_+^(2/3)) - (1 - A) |j|^2 / (2 rho^2), A_vec = (1 - A) j / rho.
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_gen3d(
    const double* __restrict__ dens_part, const double* __restrict__ jpart, int ngroups, int jgroups, int64_t M,
    FunParams fp, double Aconst, const double* __restrict__ lam, const double* __restrict__ vext,
    double* __restrict__ rho, double* __restrict__ nu, double* __restrict__ jc, double* __restrict__ U,
    double* __restrict__ delta, R* __restrict__ hA, cpx<R>* __restrict__ hD, R* __restrict__ hAx,
    R* __restrict__ hAy, R* __restrict__ hAz, int update_fields) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double sr = 0.0, snr = 0.0, sni = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const double* p = dens_part + int64_t(g) * 3 * M;
    sr += p[r];
    snr += p[M + r];
    sni += p[2 * M + r];
  }
  for (int g = 0; g < jgroups; ++g) {
    const double* q = jpart + int64_t(g) * 3 * M;
    jx += q[r];
    jy += q[M + r];
    jz += q[2 * M + r];
  }
  sr *= fp.ainv, snr *= fp.ainv, sni *= fp.ainv, jx *= fp.ainv, jy *= fp.ainv, jz *= fp.ainv;
  rho[r] = sr;
  nu[2 * r] = snr;
  nu[2 * r + 1] = sni;
  jc[r] = jx;
  jc[M + r] = jy;
  jc[2 * M + r] = jz;
  if (!update_fields) return;
  const double rp = fmax(2.0 * sr, 1e-14);
  const double gg = 1.0 / (cbrt(rp) / fp.C - lam[r]);
  const double dr = -gg * snr, di = -gg * sni;
  const double ef = 0.5 * pow(3.0 * kPi * kPi * (2.0 * sr), 2.0 / 3.0);
  const double c23 = cbrt(rp);
  const double rs = fmax(sr, 0.5e-14), cA = 1.0 - Aconst;
  const double jsq = jx * jx + jy * jy + jz * jz;
  const double u = fp.B * ef - (dr * dr + di * di) / (3.0 * fp.C * c23 * c23) - cA * jsq / (2.0 * rs * rs);
  U[r] = u;
  delta[2 * r] = dr;
  delta[2 * r + 1] = di;
  hA[r] = R(u + vext[r] - fp.mu);
  hD[r] = cpx<R>{R(dr + fp.dext[2 * r]), R(di + fp.dext[2 * r + 1])};
  hAx[r] = R(cA * jx / rs);
  hAy[r] = R(cA * jy / rs);
  hAz[r] = R(cA * jz / rs);
}

// lap f of a real field by the D2 circulants of the three axes (Eq. D2 in
// real space; c2x[m] = (D2_x)_{i, i-m}), and f converted to the context
// precision: one thread per site
template <typename R>
__global__ void k_field_lap3d(int nx, int ny, int nz, const double* __restrict__ f, const double* __restrict__ c2x,
                              const double* __restrict__ c2y, const double* __restrict__ c2z, R* __restrict__ fout,
                              R* __restrict__ lap) {
  const int64_t M = int64_t(nx) * ny * nz;
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  const int x = int(r / (int64_t(ny) * nz)), rem = int(r - int64_t(x) * ny * nz), y = rem / nz, z = rem - y * nz;
  double acc = 0.0;
  for (int q = 0; q < nx; ++q) acc += c2x[((x - q) % nx + nx) % nx] * f[(int64_t(q) * ny + y) * nz + z];
  for (int q = 0; q < ny; ++q) acc += c2y[((y - q) % ny + ny) % ny] * f[(int64_t(x) * ny + q) * nz + z];
  for (int q = 0; q < nz; ++q) acc += c2z[((z - q) % nz + nz) % nz] * f[(int64_t(x) * ny + y) * nz + q];
  lap[r] = R(acc);
  fout[r] = R(f[r]);
}

// ---------------------------------------------------------------------------
// Quantum friction on the full 3D lattice (the dissipative fields of Sec.
// 5.2, correcting the initial state by a time-dependent approach):
//   U_diss = -(alpha / rho0) div j,
//   Delta_diss = Delta [beta sin(theta_nu - theta_B') + i gamma (N - N_req) / N_req],
//   B' = -1/2 sum_n (f_v - f_u) [u lap v^* + v^* lap u]  (lap: full D2 Laplacian).
// j comes from k_jline; B' from one line pass per axis (the Laplacian is the
// sum of the per-axis D2), summed over groups; div j from line passes over
// the summed current field.

// B'_AXIS group partials over DG states, bpart[g][re|im][site] (AXIS 0
// writes, the other axes add):  -1/2 (f_v - f_u) [u (D2 v)^* + v^* D2 u]
// A lane pair per line (lane parity b: samples 2j + b).
//   grid = (ceil(NLINES / (TBG / 2)), number of groups), block = TBG
template <typename R, int NX, int NY, int NZ, int AXIS, int TBG, int DG>
__global__ __launch_bounds__(TBG) void k_bpline(const cpx<R>* __restrict__ X, int64_t nstates,
                                                const double* __restrict__ scale, const double* __restrict__ wu,
                                                const double* __restrict__ wv, double kscale2,
                                                double* __restrict__ bpart) {
  using LG = LineGeo<NX, NY, NZ, AXIS>;
  constexpr int NL = LG::NL, ST = LG::STRIDE, HL = NL / 2;
  constexpr int64_t M = int64_t(NX) * NY * NZ;
  constexpr int ES = sizeof(cpx<R>);
  const int l = blockIdx.x * (TBG / 2) + threadIdx.x / 2;
  const bool odd = threadIdx.x & 1;
  if (l >= LG::NLINES) return;  // both lanes of a pair; no barriers below
  const int s0 = LG::site0(l) + (odd ? ST : 0);
  const int64_t nbeg = int64_t(blockIdx.y) * DG;
  const int nloc = int(nstates - nbeg < DG ? nstates - nbeg : DG);
  double br[HL], bi[HL];
#pragma unroll
  for (int j = 0; j < HL; ++j) br[j] = bi[j] = 0.0;
  for (int ls = 0; ls < nloc; ++ls) {
    const int64_t n = nbeg + ls;
    const double fw = wv[n] - wu[n];
    if (fw == 0.0) continue;  // uniform over the block
    const R s = R(scale[n]);
    const bi32x4 rX = make_rsrc(X + n * 2 * M, uint32_t(2 * M * ES));
    // u (D2 v)^* first, then v^* D2 u: one transformed half-line live
    cpx<R> t[HL];
#pragma unroll 1
    for (int comp = 1; comp >= 0; --comp) {
#pragma unroll
      for (int j = 0; j < HL; ++j) t[j] = s * bload<R>(rX, s0 * ES, int(comp * M + 2 * j * ST) * ES);
      second_derivative_pair<NL>(t, R(kscale2), odd);
#pragma unroll
      for (int j = 0; j < HL; ++j) {
        if (comp == 1) {  // u (D2 v)^*
          const cpx<R> u = s * bload<R>(rX, s0 * ES, 2 * j * ST * ES);
          br[j] += -0.5 * fw * (double(u.x) * t[j].x + double(u.y) * t[j].y);
          bi[j] += -0.5 * fw * (double(u.y) * t[j].x - double(u.x) * t[j].y);
        } else {  // v^* D2 u
          const cpx<R> v = s * bload<R>(rX, s0 * ES, int(M + 2 * j * ST) * ES);
          br[j] += -0.5 * fw * (double(v.x) * t[j].x + double(v.y) * t[j].y);
          bi[j] += -0.5 * fw * (double(v.x) * t[j].y - double(v.y) * t[j].x);
        }
      }
    }
  }
  double* out = bpart + int64_t(blockIdx.y) * 2 * M + s0;
#pragma unroll
  for (int j = 0; j < HL; ++j) {
    if constexpr (AXIS == 0) {
      out[2 * j * ST] = br[j];
      out[M + 2 * j * ST] = bi[j];
    } else {
      out[2 * j * ST] += br[j];
      out[M + 2 * j * ST] += bi[j];
    }
  }
}

// per site: the current field j[3][M] and B'[M][2] from the group partials
// (fixed order) times ainv
static __global__ __launch_bounds__(256) void k_fric_sum3d(const double* __restrict__ jpart,
                                                    const double* __restrict__ bpart, int ngroups, int64_t M,
                                                    double ainv, double* __restrict__ jf, double* __restrict__ bp) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double jx = 0.0, jy = 0.0, jz = 0.0, b0 = 0.0, b1 = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const double* q = jpart + int64_t(g) * 3 * M;
    const double* b = bpart + int64_t(g) * 2 * M;
    jx += q[r];
    jy += q[M + r];
    jz += q[2 * M + r];
    b0 += b[r];
    b1 += b[M + r];
  }
  jf[r] = ainv * jx;
  jf[M + r] = ainv * jy;
  jf[2 * M + r] = ainv * jz;
  bp[2 * r] = ainv * b0;
  bp[2 * r + 1] = ainv * b1;
}

// div j: D1_AXIS (Nyquist zeroed) of the field j_AXIS = jf[AXIS][M] along its
// lines into divj (AXIS 0 writes, the other axes add); one thread per line
template <int NX, int NY, int NZ, int AXIS, int TBG>
__global__ __launch_bounds__(TBG) void k_field_d1line(const double* __restrict__ jf, double kscale,
                                                      double* __restrict__ divj) {
  using LG = LineGeo<NX, NY, NZ, AXIS>;
  constexpr int NL = LG::NL, ST = LG::STRIDE;
  constexpr int64_t M = int64_t(NX) * NY * NZ;
  const int l = blockIdx.x * TBG + threadIdx.x;
  if (l >= LG::NLINES) return;
  const int s0 = LG::site0(l);
  cpx<double> a[NL], ny;
#pragma unroll
  for (int k = 0; k < NL; ++k) a[k] = cpx<double>{jf[AXIS * M + s0 + k * ST], 0.0};
  first_derivative<NL>(a, kscale, ny);
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    if constexpr (AXIS == 0) {
      divj[s0 + k * ST] = a[k].x;
    } else {
      divj[s0 + k * ST] += a[k].x;
    }
  }
}

// N = dVe sum_r 2 rho (one workgroup, fixed order)
static __global__ __launch_bounds__(1024) void k_sum_N(int64_t M, const double* __restrict__ rho, double dVe,
                                                double* __restrict__ out) {
  __shared__ double red[1024 / kWave];
  double v = 0.0;
  for (int64_t r = threadIdx.x; r < M; r += 1024) v += 2.0 * rho[r];
  const double t = block_sum<1024>(v, red);
  if (threadIdx.x == 0) out[0] = dVe * t;
}

// the fields with the dissipative terms, one thread per site:
//   hA = U + V_ext - mu - (alpha / rho0) div j,
//   hD = Delta [1 + beta sin(theta_nu - theta_B') + i gamma (N - N_req) / N_req] + Delta_ext
template <typename R>
__global__ __launch_bounds__(256) void k_fric3d_fields(int64_t M, const double* __restrict__ divj,
                                                       const double* __restrict__ bp, const double* __restrict__ Nsum,
                                                       const double* __restrict__ nu, const double* __restrict__ U,
                                                       const double* __restrict__ delta,
                                                       const double* __restrict__ vext, const double* __restrict__ dext,
                                                       double mu, double alpha, double beta, double gamma,
                                                       double rho0, double N_req, R* __restrict__ hA,
                                                       cpx<R>* __restrict__ hD) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  const double gt = N_req > 0.0 ? gamma * (Nsum[0] - N_req) / N_req : 0.0;
  const double th_nu = atan2(nu[2 * r + 1], nu[2 * r]);
  const double th_b = atan2(bp[2 * r + 1], bp[2 * r]);
  const double fr = 1.0 + beta * sin(th_nu - th_b), fi = gt;
  const double dr = delta[2 * r], di = delta[2 * r + 1];
  hA[r] = R(U[r] + vext[r] - mu - alpha / rho0 * divj[r]);
  hD[r] = cpx<R>{R(dr * fr - di * fi + dext[2 * r]), R(dr * fi + di * fr + dext[2 * r + 1])};
}

}  // namespace tdslda
