// Static self-consistent solve of the quasi-2D problem on the device
// (Sec. 3.2, Alg. MapK; Sec. 3.1 quasi-2D item): an N_x x N_y lattice in the
// x-y plane with plane waves along z.  Every iteration builds the real BdG
// matrices of the N_z/2 + 1 distinct |k_z| (Eq. HpsiEpsi with the exact
// spectral D2 of Eq. D2 in x and y), diagonalises them in one batched
// rocSOLVER call, accumulates the T = 0 densities of the E > 0 eigenpairs
// (weighted by the |k_z| multiplicity and 1/L_z), maps them to the
// potentials (regulator with V_+ = V_ext + U_in), mixes linearly and updates
// mu for a fixed particle number (Eq. update-mu).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

namespace tdslda {

std::vector<double> spectral_d2_circulant(int N, double dz);  // q1dstatic.hip

namespace {

__global__ void k_add_shift(int M, const double* __restrict__ a, const double* __restrict__ b, double c,
                            double* __restrict__ out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < M) out[r] = a[r] + b[r] + c;
}

// H of every |k_z| class, column-major 2M x 2M (symmetric):
//   [ K + diag(hf) + kz^2/2        diag(D)               ]
//   [ diag(D)               -(K + diag(hf) + kz^2/2)     ]
// K = -1/2 (D2_x (x) 1 + 1 (x) D2_y) from the circulants d2x, d2y.
__global__ void k_st_build(double* __restrict__ H, int nclass, int nx, int ny, const double* __restrict__ kz2,
                           const double* __restrict__ hf, const double* __restrict__ dl,
                           const double* __restrict__ d2x, const double* __restrict__ d2y) {
  const int M = nx * ny, N2 = 2 * M;
  const int64_t per = int64_t(N2) * N2;
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= per * nclass) return;
  const int c = int(idx / per);
  const int rem = int(idx - int64_t(c) * per);
  const int col = rem / N2, row = rem - col * N2;
  const int ib = row / M, jb = col / M, i = row - ib * M, j = col - jb * M;
  double v = 0.0;
  if (ib == jb) {
    const int ix = i / ny, iy = i - ix * ny, jx = j / ny, jy = j - jx * ny;
    double h = 0.0;
    if (iy == jy) h += -0.5 * d2x[((ix - jx) % nx + nx) % nx];
    if (ix == jx) h += -0.5 * d2y[((iy - jy) % ny + ny) % ny];
    if (i == j) h += hf[i] + 0.5 * kz2[c];
    v = ib == 0 ? h : -h;
  } else if (i == j) {
    v = dl[i];
  }
  H[idx] = v;
}

// T = 0 densities: rho = sum_c w_c / L_z sum_{E>0} v^2 / dA,
// nu = sum_c w_c / L_z sum_{E>0} u v / dA  (real eigenvectors)
__global__ void k_st_dens(const double* __restrict__ H, const double* __restrict__ Ev, int nclass, int M,
                          const double* __restrict__ wc, double scale, double* __restrict__ rho,
                          double* __restrict__ nu) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= M) return;
  const int N2 = 2 * M;
  double sr = 0.0, sn = 0.0;
  for (int c = 0; c < nclass; ++c) {
    const double* A = H + int64_t(c) * N2 * N2;
    const double* E = Ev + int64_t(c) * N2;
    double cr = 0.0, cn = 0.0;
    for (int k = 0; k < N2; ++k) {
      if (E[k] <= 0.0) continue;
      const double u = A[int64_t(k) * N2 + r], v = A[int64_t(k) * N2 + M + r];
      cr += v * v;
      cn += u * v;
    }
    sr += wc[c] * cr;
    sn += wc[c] * cn;
  }
  rho[r] = scale * sr;
  nu[r] = scale * sn;
}

// potentials of the SLDA (A = 1) or BdG functional from rho, nu; regulator
// Lambda_c with V_+ = V_ext + U_in (k_0^2 < 0 continued analytically)
__global__ void k_st_pot(int M, const double* __restrict__ rho, const double* __restrict__ nu,
                         const double* __restrict__ vext, const double* __restrict__ Uin, double mu, double ec,
                         int kind, double B, double C, double inv_g, double* __restrict__ Uo,
                         double* __restrict__ Do, int* __restrict__ bad) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= M) return;
  const double vp = vext[r] + Uin[r];
  const double k0sq = 2.0 * (mu - vp), kcsq = 2.0 * (ec + mu - vp);
  double lam = 0.0;
  if (kcsq <= 0.0) {
    bad[0] = 1;
  } else {
    const double kc = sqrt(kcsq);
    double br;
    if (k0sq > 0.0) {
      const double k0 = sqrt(k0sq);
      br = 1.0 - k0 / (2.0 * kc) * log((kc + k0) / (kc - k0));
    } else {
      const double ka = sqrt(-k0sq);
      br = 1.0 + ka / kc * atan(ka / kc);
    }
    lam = kc / (2.0 * kPi * kPi) * br;
  }
  const double rp = fmax(2.0 * rho[r], 1e-14);
  const double ig = (kind == 1 ? cbrt(rp) / C : inv_g) - lam;
  const double d = -nu[r] / ig;
  double u = 0.0;
  if (kind == 1) {
    const double ef = 0.5 * pow(3.0 * kPi * kPi * (2.0 * rho[r]), 2.0 / 3.0);
    const double c23 = cbrt(rp);
    u = B * ef - d * d / (3.0 * C * c23 * c23);
  }
  Uo[r] = u;
  Do[r] = d;
}

// one block: N = L_z dA sum 2 rho, max |U_out - U_in|, max |D_out - D_in|
__global__ __launch_bounds__(1024) void k_st_reduce(int M, const double* __restrict__ rho,
                                                    const double* __restrict__ Uo, const double* __restrict__ Ui,
                                                    const double* __restrict__ Do, const double* __restrict__ Di,
                                                    double vol_factor, double* __restrict__ out) {
  __shared__ double sn[1024], su[1024], sd[1024];
  double n = 0.0, du = 0.0, dd = 0.0;
  for (int r = threadIdx.x; r < M; r += 1024) {
    n += 2.0 * rho[r];
    du = fmax(du, fabs(Uo[r] - Ui[r]));
    dd = fmax(dd, fabs(Do[r] - Di[r]));
  }
  sn[threadIdx.x] = n;
  su[threadIdx.x] = du;
  sd[threadIdx.x] = dd;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sn[threadIdx.x] += sn[threadIdx.x + s];
      su[threadIdx.x] = fmax(su[threadIdx.x], su[threadIdx.x + s]);
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sn[0] * vol_factor;
    out[1] = su[0];
    out[2] = sd[0];
  }
}

}  // namespace
__global__ void k_st_mix(int M, double m, const double* __restrict__ Uo, const double* __restrict__ Do,
                         double* __restrict__ U, double* __restrict__ D) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= M) return;
  U[r] = m * Uo[r] + (1.0 - m) * U[r];
  D[r] = m * Do[r] + (1.0 - m) * D[r];
}
namespace {

// Modified Broyden mixing step (one workgroup) on p = (U, Delta, mu) of
// length L = 2 M + 1, F = K[p] - p with K[p] = (U_out, Delta_out, mu_out).
// History: rows dF[k], dp[k] (k < nh, ring order) of normalised differences;
// when have_prev the difference to (pprev, Fprev) is written to row `slot`
// first (a zero row when |F - Fprev| = 0).  Then
//   a = w0^2 I + dF dF^T,  c = dF F,  gamma = a^-1 c (Cholesky, thread 0),
//   p_new = p + mix F - sum_l gamma_l (mix dF_l + dp_l),
// written over U, Delta; mu_new to out_mu.  Sums run in a fixed order.
constexpr int kBroydenMax = 8;
constexpr int kBTB = 1024;
__global__ __launch_bounds__(kBTB) void k_st_broyden(int M, double* __restrict__ U, double* __restrict__ D,
                                                     const double* __restrict__ Uo, const double* __restrict__ Do,
                                                     double mu, double mu_out, double mix, double w0, int have_prev,
                                                     int slot, int nh, double* __restrict__ pprev,
                                                     double* __restrict__ Fprev, double* __restrict__ dF,
                                                     double* __restrict__ dp, double* __restrict__ out_mu) {
  constexpr int NS = kBroydenMax * (kBroydenMax + 1) / 2 + kBroydenMax;  // a (upper) and c
  constexpr int NW = kBTB / 64;
  __shared__ double red[NW][NS];
  __shared__ double tot[NS];
  __shared__ double gam[kBroydenMax];
  const int t = threadIdx.x, L = 2 * M + 1;
  auto pval = [&](int i) { return i < M ? U[i] : (i < 2 * M ? D[i - M] : mu); };
  auto kval = [&](int i) { return i < M ? Uo[i] : (i < 2 * M ? Do[i - M] : mu_out); };
  // block sum of one value per thread (fixed order), result in tot[0]
  auto block_sum1 = [&](double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (t % 64 == 0) red[t / 64][0] = v;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[w][0];
      tot[0] = s;
    }
    __syncthreads();
    return tot[0];
  };
  if (have_prev) {
    double n2 = 0.0;
    for (int i = t; i < L; i += kBTB) {
      const double p = pval(i), F = kval(i) - p;
      const double df = F - Fprev[i];
      dF[int64_t(slot) * L + i] = df;
      dp[int64_t(slot) * L + i] = p - pprev[i];
      n2 += df * df;
    }
    // an unchanged residual gives a zero row, which takes no part in the
    // mixing (its gamma is 0)
    const double nrm = sqrt(block_sum1(n2));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = t; i < L; i += kBTB) {
      dF[int64_t(slot) * L + i] *= inv;
      dp[int64_t(slot) * L + i] *= inv;
    }
    __syncthreads();
  }
  const int nk = nh;  // rows in use (ring order)
  for (int i = t; i < L; i += kBTB) {
    const double p = pval(i);
    pprev[i] = p;
    Fprev[i] = kval(i) - p;
  }
  __syncthreads();
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  for (int i = t; i < L; i += kBTB) {
    const double F = Fprev[i];
    double f[kBroydenMax];
#pragma unroll
    for (int k = 0; k < kBroydenMax; ++k) f[k] = k < nk ? dF[int64_t(k) * L + i] : 0.0;
    int q = 0;
#pragma unroll
    for (int k = 0; k < kBroydenMax; ++k) {
#pragma unroll
      for (int l = k; l < kBroydenMax; ++l) acc[q++] += f[k] * f[l];
      acc[kBroydenMax * (kBroydenMax + 1) / 2 + k] += f[k] * F;
    }
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (t % 64 == 0) red[t / 64][q] = v;
  }
  __syncthreads();
  if (t < NS) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][t];
    tot[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    // a = w0^2 I + G (upper triangle packed row by row), Cholesky a = R^T R
    double a[kBroydenMax][kBroydenMax], c[kBroydenMax];
    int q = 0;
    for (int k = 0; k < kBroydenMax; ++k)
      for (int l = k; l < kBroydenMax; ++l) {
        a[k][l] = a[l][k] = tot[q] + (k == l ? w0 * w0 : 0.0);
        ++q;
      }
    for (int k = 0; k < kBroydenMax; ++k) c[k] = tot[kBroydenMax * (kBroydenMax + 1) / 2 + k];
    for (int j = 0; j < nk; ++j) {
      double d = a[j][j];
      for (int k = 0; k < j; ++k) d -= a[k][j] * a[k][j];
      d = sqrt(d);
      a[j][j] = d;
      for (int l = j + 1; l < nk; ++l) {
        double v = a[j][l];
        for (int k = 0; k < j; ++k) v -= a[k][j] * a[k][l];
        a[j][l] = v / d;
      }
    }
    double y[kBroydenMax];
    for (int j = 0; j < nk; ++j) {  // R^T y = c
      double v = c[j];
      for (int k = 0; k < j; ++k) v -= a[k][j] * y[k];
      y[j] = v / a[j][j];
    }
    for (int j = nk - 1; j >= 0; --j) {  // R gamma = y
      double v = y[j];
      for (int k = j + 1; k < nk; ++k) v -= a[j][k] * gam[k];
      gam[j] = v / a[j][j];
    }
  }
  __syncthreads();
  for (int i = t; i < L; i += kBTB) {
    const double F = Fprev[i];
    double v = pprev[i] + mix * F;
    for (int l = 0; l < nk; ++l) v -= gam[l] * (mix * dF[int64_t(l) * L + i] + dp[int64_t(l) * L + i]);
    if (i < M)
      U[i] = v;
    else if (i < 2 * M)
      D[i - M] = v;
    else
      *out_mu = v;
  }
}

// Fourier interpolation between two lattices of one periodic x-y box
// (Sec. 5.2, refining lattice resolution).  Positions are measured from the
// shared box corner (site i at i d); k grid of Sec. 3.1 (Nyquist at -pi/d).
__device__ __forceinline__ double kgrid_at(int l, int n, double d) {
  return 2.0 * kPi / (n * d) * double(l < n / 2 ? l : l - n);
}

// f~_lm = dx dy sum_ij f_ij exp[-2 pi i (l i / nx + m j / ny)], one thread
// per (l, m); the phase index is reduced modulo n in integers
__global__ void k_interp_coef(int nx, int ny, double dx, double dy, const double* __restrict__ f,
                              double* __restrict__ ft) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nx * ny) return;
  const int l = q / ny, m = q - l * ny;
  double re = 0.0, im = 0.0;
  for (int i = 0; i < nx; ++i) {
    const int pi_ = int((int64_t(l) * i) % nx);
    for (int j = 0; j < ny; ++j) {
      const int pj = int((int64_t(m) * j) % ny);
      const double ang = -2.0 * kPi * (double(pi_) / nx + double(pj) / ny);
      double sn, cs;
      sincos(ang, &sn, &cs);
      const double v = f[i * ny + j];
      re += v * cs;
      im += v * sn;
    }
  }
  ft[2 * q] = dx * dy * re;
  ft[2 * q + 1] = dx * dy * im;
}

// out_ab = Re 1/(Lx Ly) sum_lm f~_lm exp[i (k_l x_a + k_m y_b)], one thread per
// target site
__global__ void k_interp_eval(int nx, int ny, double dx, double dy, const double* __restrict__ ft, int nx2,
                              int ny2, double dx2, double dy2, double* __restrict__ out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nx2 * ny2) return;
  const int a = q / ny2, b = q - a * ny2;
  const double x = a * dx2, y = b * dy2;
  double acc = 0.0;
  for (int l = 0; l < nx; ++l) {
    const double kx = kgrid_at(l, nx, dx);
    for (int m = 0; m < ny; ++m) {
      double sn, cs;
      sincos(kx * x + kgrid_at(m, ny, dy) * y, &sn, &cs);
      const int c = l * ny + m;
      acc += ft[2 * c] * cs - ft[2 * c + 1] * sn;
    }
  }
  out[q] = acc / (nx * dx * ny * dy);
}

struct Handle {
  rocblas_handle h = nullptr;
  Handle() {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Fail{TDSLDA_EDEVICE, "rocblas_create_handle failed"};
  }
  ~Handle() {
    if (h) rocblas_destroy_handle(h);
  }
};

}  // namespace

// One solver instance: device buffers for a geometry, reused over iterations.
struct StaticSolver {
  const tdslda_static s;
  const tdslda_functional f;
  int M = 0, N2 = 0, nclass = 0, nyl = 1;
  double vol_factor = 1.0;
  std::vector<void*> owned;
  double *H = nullptr, *Ev = nullptr, *Ew = nullptr, *kz2 = nullptr, *wc = nullptr, *d2x = nullptr, *d2y = nullptr;
  double *vext = nullptr, *U = nullptr, *D = nullptr, *Uo = nullptr, *Do = nullptr, *hf = nullptr;
  double *rho = nullptr, *nu = nullptr, *red = nullptr;
  // Broyden mixing: previous p and F, history rows, new mu
  double *pprev = nullptr, *Fprev = nullptr, *bdF = nullptr, *bdp = nullptr, *bmu = nullptr;
  int* bad = nullptr;
  rocblas_int* info = nullptr;
  Handle rb;

  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{TDSLDA_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed (static solve)"};
    }
    owned.push_back(p);
    return p;
  }
  StaticSolver(const tdslda_static& s_, const tdslda_functional& f_, const double* vext_h) : s(s_), f(f_) {
    try {
      setup(vext_h);
    } catch (...) {
      (void)hipDeviceSynchronize();
      for (void* p : owned) (void)hipFree(p);
      owned.clear();
      throw;
    }
  }
  void setup(const double* vext_h) {
    require(s.nx > 0 && s.ny > 0 && s.nz > 0 && s.nz % 2 == 0 && s.nx % 2 == 0 && s.ny % 2 == 0, TDSLDA_EINVAL,
            "static lattice sizes must be positive and even");
    require(s.dx > 0 && s.dy > 0 && s.dz > 0 && s.ec > 0 && s.mix > 0 && s.mix <= 1, TDSLDA_EINVAL,
            "bad static solver parameters");
    require(f.functional == TDSLDA_FUNC_SLDA || f.functional == TDSLDA_FUNC_BDG, TDSLDA_EINVAL, "unknown functional");
    require(s.broyden >= 0 && s.broyden <= kBroydenMax && (s.broyden == 0 || s.w0 > 0), TDSLDA_EINVAL,
            "Broyden history must be in [0, 8] with w0 > 0");
    require(s.q1d == 0 || s.q1d == 1, TDSLDA_EINVAL, "q1d must be 0 or 1");
    // quasi-1D: the y lattice is one site; y carries plane waves instead
    nyl = s.q1d ? 1 : s.ny;
    M = s.nx * nyl;
    N2 = 2 * M;
    nclass = s.q1d ? (s.ny / 2 + 1) * (s.nz / 2 + 1) : s.nz / 2 + 1;
    // measure of a lattice site times the length of the plane-wave directions
    vol_factor = s.q1d ? s.dx * (s.ny * s.dy) * (s.nz * s.dz) : s.nz * s.dz * s.dx * s.dy;
    H = (double*)alloc(sizeof(double) * size_t(N2) * N2 * nclass);
    Ev = (double*)alloc(sizeof(double) * size_t(N2) * nclass);
    Ew = (double*)alloc(sizeof(double) * size_t(N2) * nclass);
    info = (rocblas_int*)alloc(sizeof(rocblas_int) * nclass);
    kz2 = (double*)alloc(sizeof(double) * nclass);
    wc = (double*)alloc(sizeof(double) * nclass);
    d2x = (double*)alloc(sizeof(double) * s.nx);
    d2y = (double*)alloc(sizeof(double) * nyl);
    for (double** p : {&vext, &U, &D, &Uo, &Do, &hf, &rho, &nu}) *p = (double*)alloc(sizeof(double) * M);
    red = (double*)alloc(sizeof(double) * 4);
    bad = (int*)alloc(sizeof(int));
    if (s.broyden > 0) {
      const size_t L = size_t(2 * M + 1);
      pprev = (double*)alloc(sizeof(double) * L);
      Fprev = (double*)alloc(sizeof(double) * L);
      bdF = (double*)alloc(sizeof(double) * L * s.broyden);
      bdp = (double*)alloc(sizeof(double) * L * s.broyden);
      bmu = (double*)alloc(sizeof(double));
    }
    std::vector<double> k2(nclass), w(nclass);
    auto mult = [](int m, int n) { return (m == 0 || m == n / 2) ? 1.0 : 2.0; };
    if (s.q1d) {  // classes (|k_y|, |k_z|), k_perp^2 = k_y^2 + k_z^2, multiplicity w_y w_z
      const int ncz = s.nz / 2 + 1;
      for (int my = 0; my <= s.ny / 2; ++my)
        for (int mz = 0; mz <= s.nz / 2; ++mz) {
          const double ky = 2.0 * kPi * my / (s.ny * s.dy), kz = 2.0 * kPi * mz / (s.nz * s.dz);
          k2[my * ncz + mz] = ky * ky + kz * kz;
          w[my * ncz + mz] = mult(my, s.ny) * mult(mz, s.nz);
        }
    } else {
      for (int m = 0; m < nclass; ++m) {
        const double k = 2.0 * kPi * m / (s.nz * s.dz);
        k2[m] = k * k;
        w[m] = mult(m, s.nz);
      }
    }
    const auto cx = spectral_d2_circulant(s.nx, s.dx);
    const auto cy = s.q1d ? std::vector<double>(1, 0.0) : spectral_d2_circulant(s.ny, s.dy);
    HIPCHK(hipMemcpy(kz2, k2.data(), sizeof(double) * nclass, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(wc, w.data(), sizeof(double) * nclass, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d2x, cx.data(), sizeof(double) * s.nx, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d2y, cy.data(), sizeof(double) * nyl, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(vext, vext_h, sizeof(double) * M, hipMemcpyHostToDevice));
  }
  ~StaticSolver() {
    (void)hipDeviceSynchronize();
    for (void* p : owned) (void)hipFree(p);
  }

  // K[p] for the potentials in U, D at mu: Uo, Do, rho, nu and
  // red = {N, max|dU|, max|dD|}
  void map(double mu) {
    const unsigned gb = cdiv(M, 256);
    hipLaunchKernelGGL(k_add_shift, dim3(gb), dim3(256), 0, 0, M, vext, U, -mu, hf);
    HIPCHK(hipGetLastError());
    const int64_t per = int64_t(N2) * N2;
    hipLaunchKernelGGL(k_st_build, dim3(cdiv(per * nclass, 256)), dim3(256), 0, 0, H, nclass, s.nx, nyl, kz2, hf,
                       D, d2x, d2y);
    HIPCHK(hipGetLastError());
    const rocblas_status rs = rocsolver_dsyevd_strided_batched(rb.h, rocblas_evect_original, rocblas_fill_lower, N2,
                                                               H, N2, per, Ev, N2, Ew, N2, info, nclass);
    require(rs == rocblas_status_success, TDSLDA_EDEVICE, "rocsolver_dsyevd_strided_batched failed");
    const double scale = 1.0 / vol_factor;
    hipLaunchKernelGGL(k_st_dens, dim3(gb), dim3(256), 0, 0, H, Ev, nclass, M, wc, scale, rho, nu);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemset(bad, 0, sizeof(int)));
    hipLaunchKernelGGL(k_st_pot, dim3(gb), dim3(256), 0, 0, M, rho, nu, vext, U, mu, s.ec, f.functional, f.B, f.C,
                       f.inv_g_bdg, Uo, Do, bad);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_st_reduce, dim3(1), dim3(1024), 0, 0, M, rho, Uo, U, Do, D, vol_factor, red);
    HIPCHK(hipGetLastError());
    std::vector<rocblas_int> ih(nclass);
    int b = 0;
    HIPCHK(hipMemcpy(ih.data(), info, sizeof(rocblas_int) * nclass, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&b, bad, sizeof(int), hipMemcpyDeviceToHost));
    for (int c = 0; c < nclass; ++c) require(ih[c] == 0, TDSLDA_EDEVICE, "eigensolver did not converge");
    require(b == 0, TDSLDA_EUNSTABLE, "regulator undefined (E_c + mu - V_+ <= 0 somewhere)");
  }
};

}  // namespace tdslda

// ============================================================================
// Allocation-free interpolation: the Fourier coefficients live in a fixed
// device array instead of a per-call allocation.  Each GPU the library runs
// on holds its own copy (2 x kInterpScratchPoints doubles, 1 MiB) until the
// process ends; its address is looked up once per device and only that
// address is handed to kernels (the array's name is a host-side stand-in).
constexpr int64_t kInterpScratchPoints = 65536;  // largest source lattice nx*ny
static __device__ __align__(256) double scratch[2 * kInterpScratchPoints];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up on first use)
double* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    throw tdslda::Fail{TDSLDA_EDEVICE, "no current HIP device"};
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw tdslda::Fail{TDSLDA_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e)};
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// ============================================================================
// C ABI
using tdslda::Fail;
using tdslda::StaticSolver;

extern "C" {

static tdslda_status static_guard(const char* who, const std::function<void()>& f) {
  try {
    f();
    return TDSLDA_OK;
  } catch (const Fail& e) {
    std::fprintf(stderr, "%s: %s\n", who, e.msg.c_str());
    return e.st;
  } catch (const std::bad_alloc&) {
    return TDSLDA_ENOMEM;
  } catch (...) {
    return TDSLDA_EDEVICE;
  }
}

tdslda_status tdslda_static_map(const tdslda_static* s, const tdslda_functional* fun, const double* vext,
                                const double* U, const double* delta, double mu, double* U_out,
                                double* delta_out, double* rho, double* nu, double* N) {
  if (!s || !fun || !vext || !U || !delta) return TDSLDA_EINVAL;
  return static_guard("tdslda_static_map", [&] {
    StaticSolver S(*s, *fun, vext);
    const size_t b = sizeof(double) * S.M;
    HIPCHK(hipMemcpy(S.U, U, b, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.D, delta, b, hipMemcpyHostToDevice));
    S.map(mu);
    double red[3];
    HIPCHK(hipMemcpy(red, S.red, sizeof(red), hipMemcpyDeviceToHost));
    if (U_out) HIPCHK(hipMemcpy(U_out, S.Uo, b, hipMemcpyDeviceToHost));
    if (delta_out) HIPCHK(hipMemcpy(delta_out, S.Do, b, hipMemcpyDeviceToHost));
    if (rho) HIPCHK(hipMemcpy(rho, S.rho, b, hipMemcpyDeviceToHost));
    if (nu) HIPCHK(hipMemcpy(nu, S.nu, b, hipMemcpyDeviceToHost));
    if (N) *N = red[0];
  });
}

tdslda_status tdslda_static_solve(const tdslda_static* s, const tdslda_functional* fun, const double* vext,
                                  double* U, double* delta, double* mu, int* iters, int* converged,
                                  double* hist) {
  if (!s || !fun || !vext || !U || !delta || !mu) return TDSLDA_EINVAL;
  return static_guard("tdslda_static_solve", [&] {
    require(s->maxit > 0 && s->tol > 0 && s->eF_ref > 0, TDSLDA_EINVAL, "bad iteration parameters");
    const bool fixed_n = s->a_mu != 0.0;
    require(!fixed_n || s->N_req > 0, TDSLDA_EINVAL, "fixed-N mode needs N_req > 0");
    StaticSolver S(*s, *fun, vext);
    const size_t b = sizeof(double) * S.M;
    HIPCHK(hipMemcpy(S.U, U, b, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.D, delta, b, hipMemcpyHostToDevice));
    double m = *mu;
    int done = 0, it = 0;
    for (it = 1; it <= s->maxit; ++it) {
      S.map(m);
      double red[3];
      HIPCHK(hipMemcpy(red, S.red, sizeof(red), hipMemcpyDeviceToHost));
      const double r = std::max(red[1], red[2]) / s->eF_ref;
      const double rn = fixed_n ? std::fabs(red[0] - s->N_req) / s->N_req : 0.0;
      if (hist) {
        hist[4 * (it - 1) + 0] = r;
        hist[4 * (it - 1) + 1] = rn;
        hist[4 * (it - 1) + 2] = m;
        hist[4 * (it - 1) + 3] = red[0];
      }
      require(std::isfinite(r) && std::isfinite(red[0]), TDSLDA_EUNSTABLE, "non-finite residual");
      if (r < s->tol && rn < s->tol) {
        HIPCHK(hipMemcpy(U, S.Uo, b, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(delta, S.Do, b, hipMemcpyDeviceToHost));
        done = 1;
        break;
      }
      const double mu_out = fixed_n ? m + s->a_mu / s->N_req * (s->N_req - red[0]) : m;
      if (s->broyden > 0) {
        // p = (U, Delta, mu); the difference to the previous iterate goes to
        // ring row (it - 2) mod m from the second iteration on
        const int have_prev = it > 1 ? 1 : 0;
        const int stored = it - 1;  // differences after this step
        const int slot = have_prev ? (stored - 1) % s->broyden : 0;
        const int nh = std::min(stored, s->broyden);
        hipLaunchKernelGGL(tdslda::k_st_broyden, dim3(1), dim3(tdslda::kBTB), 0, 0, S.M, S.U, S.D, S.Uo, S.Do, m,
                           mu_out, s->mix, s->w0, have_prev, slot, nh, S.pprev, S.Fprev, S.bdF, S.bdp, S.bmu);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(&m, S.bmu, sizeof(double), hipMemcpyDeviceToHost));
      } else {
        hipLaunchKernelGGL(tdslda::k_st_mix, dim3(tdslda::cdiv(S.M, 256)), dim3(256), 0, 0, S.M, s->mix, S.Uo,
                           S.Do, S.U, S.D);
        HIPCHK(hipGetLastError());
        m = mu_out;
      }
    }
    if (!done) {
      HIPCHK(hipMemcpy(U, S.U, b, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(delta, S.D, b, hipMemcpyDeviceToHost));
      it = s->maxit;
    }
    *mu = m;
    if (iters) *iters = it;
    if (converged) *converged = done;
  });
}

tdslda_status tdslda_interp2d(int nx, int ny, double dx, double dy, const double* f, int nx2, int ny2, double dx2,
                              double dy2, double* out) {
  if (!f || !out) return TDSLDA_EINVAL;
  return static_guard("tdslda_interp2d", [&] {
    require(nx > 0 && ny > 0 && nx2 > 0 && ny2 > 0 && nx % 2 == 0 && ny % 2 == 0, TDSLDA_EINVAL,
            "lattice sizes must be positive (source sizes even)");
    require(nx <= 4096 && ny <= 4096 && int64_t(nx2) * ny2 <= (int64_t(1) << 28), TDSLDA_EINVAL,
            "lattice too large for the direct sums");
    require(dx > 0 && dy > 0 && dx2 > 0 && dy2 > 0, TDSLDA_EINVAL, "spacings must be positive");
    const double Lx = nx * dx, Ly = ny * dy;
    require(std::fabs(nx2 * dx2 - Lx) <= 1e-12 * Lx && std::fabs(ny2 * dy2 - Ly) <= 1e-12 * Ly, TDSLDA_EINVAL,
            "the two lattices must span the same box");
    const size_t n1 = size_t(nx) * ny, n2 = size_t(nx2) * ny2;
    double *df = nullptr, *dft = nullptr, *dout = nullptr;
    auto release = [&] {
      if (df) (void)hipFree(df);
      if (dft) (void)hipFree(dft);
      if (dout) (void)hipFree(dout);
    };
    if (hipMalloc(&df, n1 * sizeof(double)) != hipSuccess || hipMalloc(&dft, 2 * n1 * sizeof(double)) != hipSuccess ||
        hipMalloc(&dout, n2 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      release();
      throw Fail{TDSLDA_ENOMEM, "hipMalloc failed (interp2d)"};
    }
    try {
      HIPCHK(hipMemcpy(df, f, n1 * sizeof(double), hipMemcpyHostToDevice));
      hipLaunchKernelGGL(tdslda::k_interp_coef, dim3(tdslda::cdiv(int64_t(n1), 256)), dim3(256), 0, 0, nx, ny, dx,
                         dy, df, dft);
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(tdslda::k_interp_eval, dim3(tdslda::cdiv(int64_t(n2), 256)), dim3(256), 0, 0, nx, ny, dx,
                         dy, dft, nx2, ny2, dx2, dy2, dout);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpy(out, dout, n2 * sizeof(double), hipMemcpyDeviceToHost));
    } catch (...) {
      (void)hipDeviceSynchronize();
      release();
      throw;
    }
    release();
  });
}

tdslda_status tdslda_interp2d_noalloc(int nx, int ny, double dx, double dy, const double* f_dev, int nx2, int ny2,
                                      double dx2, double dy2, double* out_dev, void* hip_stream) {
  if (!f_dev || !out_dev) return TDSLDA_EINVAL;
  return static_guard("tdslda_interp2d_noalloc", [&] {
    require(nx > 0 && ny > 0 && nx2 > 0 && ny2 > 0 && nx % 2 == 0 && ny % 2 == 0, TDSLDA_EINVAL,
            "lattice sizes must be positive (source sizes even)");
    require(int64_t(nx) * ny <= kInterpScratchPoints, TDSLDA_EINVAL,
            "source lattice larger than the fixed coefficient array (nx * ny <= 65536)");
    require(int64_t(nx2) * ny2 <= (int64_t(1) << 28), TDSLDA_EINVAL, "target lattice too large for the direct sums");
    require(dx > 0 && dy > 0 && dx2 > 0 && dy2 > 0, TDSLDA_EINVAL, "spacings must be positive");
    const double Lx = nx * dx, Ly = ny * dy;
    require(std::fabs(nx2 * dx2 - Lx) <= 1e-12 * Lx && std::fabs(ny2 * dy2 - Ly) <= 1e-12 * Ly, TDSLDA_EINVAL,
            "the two lattices must span the same box");
    double* ft = scratch_on_current_device();
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t n1 = int64_t(nx) * ny, n2 = int64_t(nx2) * ny2;
    hipLaunchKernelGGL(tdslda::k_interp_coef, dim3(tdslda::cdiv(n1, 256)), dim3(256), 0, st, nx, ny, dx, dy, f_dev,
                       ft);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(tdslda::k_interp_eval, dim3(tdslda::cdiv(n2, 256)), dim3(256), 0, st, nx, ny, dx, dy, ft, nx2,
                       ny2, dx2, dy2, out_dev);
    HIPCHK(hipGetLastError());
  });
}

}  // extern "C"
