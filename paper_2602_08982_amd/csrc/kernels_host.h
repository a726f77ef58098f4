// Non-template kernels used only by the C-ABI translation unit: per-state
// scalar finalisation, gradient-density reduction, energy terms and set-up.
#pragma once

#include "kernels3d.h"

namespace tdslda {

// finalize per-state scalars
// (norm^2 = dV sum |phi|^2; the partials hold the plain sums).  <H>_n: the
// first n_raw h slots hold partials of the stored (unscaled) state and are
// multiplied by scale^2; the others are already on the normalised state.
__global__ void k_finalize(int64_t nstates, StateScalars sc, int n_nrm, int n_h, int n_raw, int do_scale,
                           int do_h, double dV) {
  const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (n >= nstates) return;
  if (do_scale) {
    double s = 0.0;
    for (int i = 0; i < n_nrm; ++i) s += sc.nrm_part[n * sc.nrm_stride + i];
    sc.scale[n] = 1.0 / sqrt(dV * s);
  }
  if (do_h) {
    double r = 0.0, s = 0.0;
    for (int i = 0; i < n_raw; ++i) r += sc.h_part[n * sc.h_stride + i];
    for (int i = n_raw; i < n_h; ++i) s += sc.h_part[n * sc.h_stride + i];
    const double sn = sc.scale[n];
    sc.hshift[n] = sn * sn * r + s;
  }
}

// sum the per-state scratch over the chunk (fixed order) into tau, j
__global__ void k_grad_reduce(int64_t nchunk, int64_t M, double ainv, const double* __restrict__ tau_s,
                              const double* __restrict__ j_s, double* __restrict__ tau,
                              double* __restrict__ j, int init) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double t = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) {
    t += tau_s[c * M + r];
    jx += j_s[(c * 3 + 0) * M + r];
    jy += j_s[(c * 3 + 1) * M + r];
    jz += j_s[(c * 3 + 2) * M + r];
  }
  if (init) {
    tau[r] = ainv * t;
    j[r] = ainv * jx;
    j[M + r] = ainv * jy;
    j[2 * M + r] = ainv * jz;
  } else {
    tau[r] += ainv * t;
    j[r] += ainv * jx;
    j[M + r] += ainv * jy;
    j[2 * M + r] += ainv * jz;
  }
}

// ---------------------------------------------------------------------------
// Energy terms of Sec. 3.2 (A = 1, spin-symmetric) reduced in one block:
// out = {E_kin, E_pot, E_pair, E_curr, E_ext, N, E_pair.ext}
// with E_pair.ext = -int (Delta_ext nu^* + c.c.)
__global__ __launch_bounds__(1024) void k_energy(int64_t M, const double* __restrict__ rho,
                                                 const double* __restrict__ tau,
                                                 const double* __restrict__ nu,
                                                 const double* __restrict__ j,
                                                 const double* __restrict__ delta,
                                                 const double* __restrict__ vext,
                                                 const double* __restrict__ dext, double B, double A,
                                                 int slda, double dVe, double* __restrict__ out) {
  __shared__ double red[1024 / kWave];
  double ek = 0, ep = 0, epa = 0, ec = 0, ee = 0, nn = 0, epx = 0;
  for (int64_t r = threadIdx.x; r < M; r += 1024) {
    const double rs = fmax(rho[r], 0.5e-14);
    const double jsq = j[r] * j[r] + j[M + r] * j[M + r] + j[2 * M + r] * j[2 * M + r];
    ek += A * (tau[r] - jsq / rs);
    if (slda) ep += 0.6 * B * (2.0 * rho[r]) * 0.5 * pow(3.0 * kPi * kPi * (2.0 * rho[r]), 2.0 / 3.0);
    epa -= delta[2 * r] * nu[2 * r] + delta[2 * r + 1] * nu[2 * r + 1];
    ec += jsq / rs;
    ee += vext[r] * 2.0 * rho[r];
    nn += 2.0 * rho[r];
    epx -= 2.0 * (dext[2 * r] * nu[2 * r] + dext[2 * r + 1] * nu[2 * r + 1]);
  }
  double v[7] = {ek, ep, epa, ec, ee, nn, epx};
  for (int k = 0; k < 7; ++k) {
    const double t = block_sum<1024>(v[k], red);
    if (threadIdx.x == 0) out[k] = t * dVe;
  }
}

// Energy terms of the spin-imbalanced ASLDA functional (Sec. 2.4) from the
// spin-resolved densities ([spin][M]: rho, tau; j [spin][3][M]; nu [M][2]; Delta as
// built): E_kin = sum_s A_s/2 (tau_s - j_s^2/rho_s), E_pot = 3/5 B rho_+ eF,
// E_pair = -Re Delta^* nu, E_curr = sum_s j_s^2 / (2 rho_s), E_ext =
// V_ext rho_+, rho_+, E_pair.ext, each times dVe; out[7] = N_a, out[8] = N_b.
__device__ __forceinline__ double host_aslda_A(double p) {
  const double p2 = p * p;
  return 1.094 + 0.156 * p * (1.0 - 2.0 * p2 / 3.0 + p2 * p2 / 5.0) - 0.532 * p2 * (1.0 - p2 + p2 * p2 / 3.0);
}
__global__ __launch_bounds__(1024) void k_energy_aslda(int64_t M, const double* __restrict__ rho,
                                                       const double* __restrict__ tau,
                                                       const double* __restrict__ nu,
                                                       const double* __restrict__ j,
                                                       const double* __restrict__ delta,
                                                       const double* __restrict__ vext,
                                                       const double* __restrict__ dext, double dVe,
                                                       double* __restrict__ out) {
  __shared__ double red[1024 / kWave];
  double ek = 0, ep = 0, epa = 0, ec = 0, ee = 0, nn = 0, epx = 0, na = 0, nb = 0;
  for (int64_t r = threadIdx.x; r < M; r += 1024) {
    const double ra = fmax(rho[r], 0.5e-14), rb = fmax(rho[M + r], 0.5e-14), rp = ra + rb;
    const double p = (ra - rb) / rp;
    const double Aa = host_aslda_A(p), Ab = host_aslda_A(-p);
    const double hp = 0.5 * (1.0 + p), hm = 0.5 * (1.0 - p);
    const double B = 1.5874010519681994 * (0.357 + 0.642 * p * p - Aa * pow(hp, 5.0 / 3.0) - Ab * pow(hm, 5.0 / 3.0));
    double jsa = 0.0, jsb = 0.0;
    for (int c = 0; c < 3; ++c) {
      jsa += j[c * M + r] * j[c * M + r];
      jsb += j[(3 + c) * M + r] * j[(3 + c) * M + r];
    }
    ek += 0.5 * Aa * (tau[r] - jsa / ra) + 0.5 * Ab * (tau[M + r] - jsb / rb);
    ep += 0.6 * B * rp * 0.5 * pow(3.0 * kPi * kPi * rp, 2.0 / 3.0);
    epa -= delta[2 * r] * nu[2 * r] + delta[2 * r + 1] * nu[2 * r + 1];
    ec += jsa / (2.0 * ra) + jsb / (2.0 * rb);
    ee += vext[r] * (rho[r] + rho[M + r]);
    nn += rho[r] + rho[M + r];
    na += rho[r];
    nb += rho[M + r];
    epx -= 2.0 * (dext[2 * r] * nu[2 * r] + dext[2 * r + 1] * nu[2 * r + 1]);
  }
  double v[9] = {ek, ep, epa, ec, ee, nn, epx, na, nb};
  for (int k = 0; k < 9; ++k) {
    const double t = block_sum<1024>(v[k], red);
    if (threadIdx.x == 0) out[k] = t * dVe;
  }
}

// ---------------------------------------------------------------------------
// Streaming copy: each thread moves CP_U 16-byte words with non-temporal
// 128-bit loads and stores; consecutive lanes touch consecutive words.
constexpr int CP_TB = 256, CP_U = 4;
typedef int cp_v4i __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(CP_TB) void k_stream_copy(const cp_v4i* __restrict__ src, cp_v4i* __restrict__ dst,
                                                       int64_t n16) {
  const int64_t base = int64_t(blockIdx.x) * (CP_TB * CP_U) + threadIdx.x;
  cp_v4i v[CP_U];
#pragma unroll
  for (int k = 0; k < CP_U; ++k) {
    const int64_t i = base + int64_t(k) * CP_TB;
    if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < CP_U; ++k) {
    const int64_t i = base + int64_t(k) * CP_TB;
    if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
  }
}

// Streaming read: each thread reads RD_U 16-byte words (non-temporal) and
// folds them with xor; the fold reaches memory only through a branch no
// ordinary data takes, which keeps every load live.  The read-only HBM
// reference of the measurement.
constexpr int RD_TB = 256, RD_U = 8;
__global__ __launch_bounds__(RD_TB) void k_stream_read(const cp_v4i* __restrict__ src, cp_v4i* __restrict__ sink,
                                                       int64_t n16) {
  const int64_t base = int64_t(blockIdx.x) * (RD_TB * RD_U) + threadIdx.x;
  cp_v4i x = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < RD_U; ++k) {
    const int64_t i = base + int64_t(k) * RD_TB;
    if (i < n16) x ^= __builtin_nontemporal_load(src + i);
  }
  if (x.x == 0x7fffffff && x.y == 0x7ffffffe && x.z == 0x7ffffffd && x.w == 0x7ffffffc) sink[0] = x;
}

// ---------------------------------------------------------------------------
// set-up kernels
// Lambda_c of Eq. Creg with V_+ = vext (A = 1); k_0^2 < 0 continued
// analytically (k_0 = i kappa).
__global__ void k_lambda(int64_t M, const double* __restrict__ vext, double mu, double ec, double A,
                         double* __restrict__ lam, int* __restrict__ bad) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  const double k0sq = 2.0 * (mu - vext[r]) / A;
  const double kcsq = 2.0 * (ec + mu - vext[r]) / A;
  if (kcsq <= 0.0) {
    bad[0] = 1;
    lam[r] = 0.0;
    return;
  }
  const double kc = sqrt(kcsq);
  double br;
  if (k0sq > 0.0) {
    const double k0 = sqrt(k0sq);
    br = 1.0 - k0 / (2.0 * kc) * log((kc + k0) / (kc - k0));
  } else {
    const double ka = sqrt(-k0sq);
    br = 1.0 + ka / kc * atan(ka / kc);
  }
  lam[r] = kc / (2.0 * kPi * kPi * A) * br;
}

// FP64 -> context precision, real field
template <typename R>
__global__ void k_convert_real(int64_t M, const double* __restrict__ in, R* __restrict__ out) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r < M) out[r] = R(in[r]);
}

// out[r] = value (the constant inverse effective mass of the functional)
template <typename R>
__global__ void k_fill_real(int64_t M, double value, R* __restrict__ out) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r < M) out[r] = R(value);
}


// theta(x, y) of straight vortex lines along z (centred coordinates)
__global__ void k_vortex_phase(int64_t M, int nx, int ny, int nz, double dx, double dy, int nv,
                               const double* __restrict__ xyq, double* __restrict__ theta) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  const int ix = int(r / (int64_t(ny) * nz)), iy = int((r / nz) % ny);
  const double x = (ix - nx / 2) * dx, y = (iy - ny / 2) * dy;
  double th = 0.0;
  for (int v = 0; v < nv; ++v) th += xyq[3 * v + 2] * atan2(y - xyq[3 * v + 1], x - xyq[3 * v]);
  theta[r] = th;
}

// Fermi weights of the frozen static energies
// times the state's multiplicity (the number of equal problems it stands
// for: the two signs of k_z of a quasi-2D class)
__global__ void k_weights(int64_t n, const double* __restrict__ E, double T, const double* __restrict__ mult,
                          double* __restrict__ wu, double* __restrict__ wv) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double e = E[i], m = mult[i];
  if (T <= 0.0) {
    wu[i] = m * (e < 0 ? 1.0 : (e > 0 ? 0.0 : 0.5));
    wv[i] = m * (e > 0 ? 1.0 : (e < 0 ? 0.0 : 0.5));
  } else {
    wu[i] = m / (exp(fmin(fmax(e / T, -700.0), 700.0)) + 1.0);
    wv[i] = m / (exp(fmin(fmax(-e / T, -700.0), 700.0)) + 1.0);
  }
}

// quasi-2D plane-wave states of the uniform H (one block row per state):
// kidx[n] = (l_x, l_y, m_z), lattice momenta k = 2 pi l / L along x, y and
// the |k_z| class m_z in [0, nkz/2] (k_z = 2 pi m_z / L_z), xi = k^2/2 +
// hshift, u = sqrt((1 + xi/E)/2), v = sqrt((1 - xi/E)/2) times
// exp(i (k_x x + k_y y)) / sqrt(L_x L_y); writes E, k_z^2 and the class
// multiplicity (1 for m_z = 0 and the Nyquist class, 2 otherwise)
template <typename R>
__global__ void k_q2_plane_waves(int64_t M, int64_t nstates, int nx, int ny, int nkz, const int32_t* __restrict__ kidx,
                                 double hshift, double delta0, double kx, double ky, double kz, double invsqrtA,
                                 cpx<R>* __restrict__ X, double* __restrict__ E, double* __restrict__ kz2,
                                 double* __restrict__ mult) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  for (int64_t n = blockIdx.y; n < nstates; n += gridDim.y) {
  const int lx = kidx[3 * n], ly = kidx[3 * n + 1], mz = kidx[3 * n + 2];
  const int mx = lx < nx / 2 ? lx : lx - nx, my = ly < ny / 2 ? ly : ly - ny;
  const double kz2n = kz * kz * mz * mz;
  const double k2 = kx * kx * mx * mx + ky * ky * my * my + kz2n;
  const double xi = 0.5 * k2 + hshift;
  const double e = sqrt(xi * xi + delta0 * delta0);
  const double uk = sqrt(0.5 * (1.0 + xi / e)), vk = sqrt(0.5 * (1.0 - xi / e));
  if (r == 0) {
    E[n] = e;
    kz2[n] = kz2n;
    mult[n] = (mz == 0 || 2 * mz == nkz) ? 1.0 : 2.0;
  }
  if (r >= M) continue;
  const int ix = int(r / ny), iy = int(r % ny);
  const long fx = (long(lx) * ix) % nx, fy = (long(ly) * iy) % ny;
  const double frac = double(fx) / nx + double(fy) / ny;
  double sn, cs;
  sincospi(2.0 * frac, &sn, &cs);
  X[n * 2 * M + r] = cpx<R>{R(uk * cs * invsqrtA), R(uk * sn * invsqrtA)};
  X[n * 2 * M + M + r] = cpx<R>{R(vk * cs * invsqrtA), R(vk * sn * invsqrtA)};
  }
}

}  // namespace tdslda
