// Static quasiparticle states of the batched quasi-1D problems: for every
// transverse momentum the 2N_z x 2N_z BdG matrix of the reduced problem
// (Sec. 2.3, Eq. HpsiEpsi; quasi-1D item of Sec. 3.1: mu -> mu - k_perp^2/2;
// the z kinetic term is the exact spectral second-derivative matrix of
// Eq. D2, Nyquist mode kept) is built on the device and diagonalised in
// batches with rocSOLVER; the eigenpairs with 0 < E < E_c are the states
// that are evolved (E > 0 half of the spin-symmetric spectrum, cutoff of the
// quasi-1D configurations).  Spin-imbalanced problems carry their own
// diagonal in each block (h_a - mu_a above, -(h_b - mu_b) below) and keep
// both branches, |E| < E_c.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ctx.h"

namespace tdslda {
namespace {

// H of problems p0 .. p0+nb-1, column-major 2N x 2N each (symmetric, so the
// storage order only fixes which triangle rocSOLVER reads):
//   [ h_a      diag(D) ]     h_s = -1/2 D2 + diag(hfield_s) + k_perp^2/2
//   [ diag(D)   -h_b   ]     (real pairing field D; hfield_b = hfield_a
//                             for the spin-symmetric problem)
__global__ void k_q1d_build(double* __restrict__ H, int nb, int p0, int N, const double* __restrict__ kp2,
                            const double* __restrict__ hfield, const double* __restrict__ hfield_b,
                            const double* __restrict__ delta, const double* __restrict__ d2) {
  const int N2 = 2 * N;
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t per = int64_t(N2) * N2;
  if (idx >= per * nb) return;
  const int b = int(idx / per);
  const int rem = int(idx - int64_t(b) * per);
  const int col = rem / N2, row = rem - col * N2;
  const int ib = row / N, jb = col / N, i = row - ib * N, j = col - jb * N;
  double v = 0.0;
  if (ib == jb) {
    const int m = ((i - j) % N + N) % N;
    double h = -0.5 * d2[m];
    if (i == j) h += (ib == 0 ? hfield[i] : hfield_b[i]) + 0.5 * kp2[p0 + b];
    v = ib == 0 ? h : -h;
  } else if (i == j) {
    v = delta[i];
  }
  H[idx] = v;
}

// copy eigenvector `col` of matrix b into state slot n (u = rows 0..N-1,
// v = rows N..2N-1), dividing by sqrt(dz) (int |phi|^2 dz = 1)
template <typename R>
__global__ void k_q1d_take(const double* __restrict__ H, const int32_t* __restrict__ jobs, int njobs, int N,
                           double inv_sqrt_dz, cpx<R>* __restrict__ X) {
  const int job = blockIdx.x;
  if (job >= njobs) return;
  const int b = jobs[3 * job], col = jobs[3 * job + 1], slot = jobs[3 * job + 2];
  const int N2 = 2 * N;
  const double* src = H + (int64_t(b) * N2 + col) * N2;
  for (int r = threadIdx.x; r < N2; r += blockDim.x)
    X[int64_t(slot) * N2 + r] = cpx<R>{R(src[r] * inv_sqrt_dz), R(0)};
}

struct Rocblas {
  rocblas_handle h = nullptr;
  explicit Rocblas(hipStream_t s) {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Fail{TDSLDA_EDEVICE, "rocblas_create_handle failed"};
    rocblas_set_stream(h, s);
  }
  ~Rocblas() {
    if (h) rocblas_destroy_handle(h);
  }
};

}  // namespace

// Exact spectral D2 along a periodic axis as a circulant: d2[m] =
// (1/N) sum_k (-k^2) cos(k m dz), k on the grid of Sec. 3.1 (Nyquist kept).
std::vector<double> spectral_d2_circulant(int N, double dz) {
  std::vector<double> d2(N, 0.0);
  for (int m = 0; m < N; ++m) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) {
      const int mj = j < N / 2 ? j : j - N;
      const double k = 2.0 * kPi * mj / (N * dz);
      s -= k * k * std::cos(2.0 * kPi * double((int64_t(j) * m) % N) / N);
    }
    d2[m] = s / N;
  }
  return d2;
}

int64_t q1d_static(hipStream_t st, int N, double dz, int nprob, const double* kperp2, const double* hfield,
                   const double* delta, double ecut, int32_t* counts, void* X, size_t esz, double* E_dev,
                   double* kp_dev, int64_t cap, const double* hfield_b, bool both) {
  const int N2 = 2 * N;
  const bool vectors = X != nullptr;
  const int64_t per = int64_t(N2) * N2;
  // batch so that the matrices take about 1 GiB
  const int B = int(std::max<int64_t>(1, std::min<int64_t>(nprob, (int64_t(1) << 30) / (per * 8))));
  Rocblas rb(st);
  std::vector<void*> owned;
  auto alloc = [&](size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      for (void* q : owned) (void)hipFree(q);
      throw Fail{TDSLDA_ENOMEM, "hipMalloc failed in the quasi-1D static solve"};
    }
    owned.push_back(p);
    return p;
  };
  double* H = (double*)alloc(sizeof(double) * per * B);
  double* D = (double*)alloc(sizeof(double) * N2 * B);
  double* Ework = (double*)alloc(sizeof(double) * N2 * B);
  rocblas_int* info = (rocblas_int*)alloc(sizeof(rocblas_int) * B);
  double* kp_d = (double*)alloc(sizeof(double) * nprob);
  double* hf_d = (double*)alloc(sizeof(double) * 2 * N);
  double* de_d = (double*)alloc(sizeof(double) * N);
  double* d2_d = (double*)alloc(sizeof(double) * N);
  int32_t* jobs_d = (int32_t*)alloc(sizeof(int32_t) * 3 * N2 * B);
  const std::vector<double> d2 = spectral_d2_circulant(N, dz);
  try {
    HIPCHK(hipMemcpyAsync(kp_d, kperp2, sizeof(double) * nprob, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(hf_d, hfield, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(hf_d + N, hfield_b ? hfield_b : hfield, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(de_d, delta, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d2_d, d2.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    std::vector<double> Dh(size_t(N2) * B);
    std::vector<rocblas_int> infoh(B);
    std::vector<int32_t> jobs;
    std::vector<double> Eh, kph;
    int64_t total = 0;
    for (int p0 = 0; p0 < nprob; p0 += B) {
      const int nb = std::min(B, nprob - p0);
      hipLaunchKernelGGL(k_q1d_build, dim3(cdiv(per * nb, 256)), dim3(256), 0, st, H, nb, p0, N, kp_d, hf_d,
                         hf_d + N, de_d, d2_d);
      HIPCHK(hipGetLastError());
      const rocblas_status rs = rocsolver_dsyevd_strided_batched(
          rb.h, vectors ? rocblas_evect_original : rocblas_evect_none, rocblas_fill_lower, N2, H, N2, per, D, N2,
          Ework, N2, info, nb);
      require(rs == rocblas_status_success, TDSLDA_EDEVICE, "rocsolver_dsyevd_strided_batched failed");
      HIPCHK(hipMemcpyAsync(Dh.data(), D, sizeof(double) * N2 * nb, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(infoh.data(), info, sizeof(rocblas_int) * nb, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      jobs.clear();
      Eh.clear();
      kph.clear();
      for (int b = 0; b < nb; ++b) {
        require(infoh[b] == 0, TDSLDA_EDEVICE, "eigensolver did not converge for problem " + std::to_string(p0 + b));
        int cnt = 0;
        for (int k = 0; k < N2; ++k) {
          const double e = Dh[size_t(b) * N2 + k];
          if (both ? std::fabs(e) < ecut : (e > 0.0 && e < ecut)) {
            if (vectors) {
              require(total < cap, TDSLDA_EINVAL, "context capacity below the number of kept states");
              jobs.push_back(b);
              jobs.push_back(k);
              jobs.push_back(int32_t(total));
              Eh.push_back(e);
              kph.push_back(kperp2[p0 + b]);
            }
            ++total;
            ++cnt;
          }
        }
        if (counts) counts[p0 + b] = cnt;
      }
      if (vectors && !jobs.empty()) {
        const int nj = int(jobs.size() / 3);
        const int64_t first = jobs[2];
        HIPCHK(hipMemcpyAsync(jobs_d, jobs.data(), sizeof(int32_t) * jobs.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(E_dev + first, Eh.data(), sizeof(double) * nj, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(kp_dev + first, kph.data(), sizeof(double) * nj, hipMemcpyHostToDevice, st));
        if (esz == 16)
          hipLaunchKernelGGL((k_q1d_take<double>), dim3(nj), dim3(256), 0, st, H, jobs_d, nj, N, 1.0 / std::sqrt(dz),
                             (cpx<double>*)X);
        else
          hipLaunchKernelGGL((k_q1d_take<float>), dim3(nj), dim3(256), 0, st, H, jobs_d, nj, N, 1.0 / std::sqrt(dz),
                             (cpx<float>*)X);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));  // jobs_d and the host vectors are reused
      }
    }
    HIPCHK(hipStreamSynchronize(st));
    for (void* q : owned) (void)hipFree(q);
    return total;
  } catch (...) {
    (void)hipStreamSynchronize(st);
    for (void* q : owned) (void)hipFree(q);
    throw;
  }
}

}  // namespace tdslda
