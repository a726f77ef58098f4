// Warm-start network of the static workflow: forward, backward and Adam in
// hand-written kernels (FP32 weights, FP32 activations).  The network maps
// the normalised external potential of an H x W x-y lattice to normalised
// self-consistent (U, Delta) maps and the chemical potential:
//   h1 = relu(conv3(x)), h2 = relu(conv3(h1)), h3 = relu(conv3(h2)),
//   maps = conv1(h3) (2 channels), mu = mean_{H,W}(h3) . w_mu + b_mu,
// conv3 = 3x3 convolution with periodic padding.  Loss
//   L = mean((maps - Y)^2) + lam_mu mean((mu - y_mu)^2).
// Flat parameter order: W1 b1 W2 b2 W3 b3 Wm bm w_mu b_mu, conv weights
// [Cout][Cin][3][3].  Every reduction is a fixed-order loop (no atomics), so
// forward and gradients are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/tdslda.h"

namespace {

struct NnFail {
  tdslda_status st;
  std::string msg;
};

#define NNCHK(x)                                                                    \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) throw NnFail{TDSLDA_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

inline unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

// y[n,o,i,j] = b[o] + sum_{c,di,dj} W[o,c,di,dj] x[n,c,i+di-1,j+dj-1]; h = relu(y)
__global__ void k_conv3_fwd(int B, int Ci, int Co, int H, int W, const float* __restrict__ x,
                            const float* __restrict__ w, const float* __restrict__ b, float* __restrict__ z,
                            float* __restrict__ h) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t tot = int64_t(B) * Co * H * W;
  if (idx >= tot) return;
  const int j = int(idx % W), i = int((idx / W) % H), o = int((idx / (int64_t(W) * H)) % Co);
  const int n = int(idx / (int64_t(W) * H * Co));
  float s = b[o];
  for (int c = 0; c < Ci; ++c) {
    const float* xc = x + (int64_t(n) * Ci + c) * H * W;
    const float* wc = w + (int64_t(o) * Ci + c) * 9;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = (i + di - 1 + H) % H;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) s += wc[di * 3 + dj] * xc[ii * W + (j + dj - 1 + W) % W];
    }
  }
  z[idx] = s;
  h[idx] = s > 0.f ? s : 0.f;
}

// maps[n,k,i,j] = bm[k] + sum_c Wm[k,c] h3[n,c,i,j]
__global__ void k_head_fwd(int B, int C, int HW, const float* __restrict__ h3, const float* __restrict__ wm,
                           const float* __restrict__ bm, float* __restrict__ maps) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(B) * 2 * HW) return;
  const int p = int(idx % HW), k = int((idx / HW) % 2), n = int(idx / (2 * int64_t(HW)));
  float s = bm[k];
  for (int c = 0; c < C; ++c) s += wm[k * C + c] * h3[(int64_t(n) * C + c) * HW + p];
  maps[idx] = s;
}

// g[n,c] = mean_p h3[n,c,p]
__global__ void k_gap(int B, int C, int HW, const float* __restrict__ h3, float* __restrict__ g) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= B * C) return;
  const float* src = h3 + int64_t(idx) * HW;
  float s = 0.f;
  for (int p = 0; p < HW; ++p) s += src[p];
  g[idx] = s / float(HW);
}

// mu[n] = sum_c g[n,c] wmu[c] + bmu
__global__ void k_mu(int B, int C, const float* __restrict__ g, const float* __restrict__ wmu,
                     const float* __restrict__ bmu, float* __restrict__ mu) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= B) return;
  float s = bmu[0];
  for (int c = 0; c < C; ++c) s += g[n * C + c] * wmu[c];
  mu[n] = s;
}

// loss and its gradients w.r.t. maps and mu (one block, fixed order)
__global__ __launch_bounds__(256) void k_loss(int B, int HW, const float* __restrict__ maps,
                                              const float* __restrict__ Y, const float* __restrict__ mu,
                                              const float* __restrict__ ymu, float lam, float* __restrict__ gmaps,
                                              float* __restrict__ gmu, float* __restrict__ loss) {
  __shared__ float red[256];
  const int64_t nm = int64_t(B) * 2 * HW;
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < nm; i += 256) {
    const float d = maps[i] - Y[i];
    s += d * d;
    gmaps[i] = 2.f * d / float(nm);
  }
  float sm = 0.f;
  for (int n = threadIdx.x; n < B; n += 256) {
    const float d = mu[n] - ymu[n];
    sm += d * d;
    gmu[n] = 2.f * lam * d / float(B);
  }
  red[threadIdx.x] = s / float(nm) + lam * sm / float(B);
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0];
}

// head gradients: gWm[k,c], gbm[k], gwmu[c], gbmu
__global__ void k_head_bwd_w(int B, int C, int HW, const float* __restrict__ gmaps, const float* __restrict__ h3,
                             const float* __restrict__ g, const float* __restrict__ gmu, float* __restrict__ gwm,
                             float* __restrict__ gbm, float* __restrict__ gwmu, float* __restrict__ gbmu) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < 2 * C) {
    const int k = idx / C, c = idx % C;
    float s = 0.f;
    for (int n = 0; n < B; ++n) {
      const float* gm = gmaps + (int64_t(n) * 2 + k) * HW;
      const float* hh = h3 + (int64_t(n) * C + c) * HW;
      for (int p = 0; p < HW; ++p) s += gm[p] * hh[p];
    }
    gwm[idx] = s;
  } else if (idx < 2 * C + 2) {
    const int k = idx - 2 * C;
    float s = 0.f;
    for (int n = 0; n < B; ++n)
      for (int p = 0; p < HW; ++p) s += gmaps[(int64_t(n) * 2 + k) * HW + p];
    gbm[k] = s;
  } else if (idx < 3 * C + 2) {
    const int c = idx - 2 * C - 2;
    float s = 0.f;
    for (int n = 0; n < B; ++n) s += g[n * C + c] * gmu[n];
    gwmu[c] = s;
  } else if (idx == 3 * C + 2) {
    float s = 0.f;
    for (int n = 0; n < B; ++n) s += gmu[n];
    gbmu[0] = s;
  }
}

// gz3 = (Wm^T gmaps + gmu wmu / HW) * [z3 > 0]
__global__ void k_head_bwd_x(int B, int C, int HW, const float* __restrict__ gmaps, const float* __restrict__ gmu,
                             const float* __restrict__ wm, const float* __restrict__ wmu,
                             const float* __restrict__ z3, float* __restrict__ gz) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(B) * C * HW) return;
  const int p = int(idx % HW), c = int((idx / HW) % C), n = int(idx / (int64_t(C) * HW));
  float s = wm[c] * gmaps[(int64_t(n) * 2) * HW + p] + wm[C + c] * gmaps[(int64_t(n) * 2 + 1) * HW + p] +
            gmu[n] * wmu[c] / float(HW);
  gz[idx] = z3[idx] > 0.f ? s : 0.f;
}

// gx[n,c,i,j] = sum_{o,di,dj} W[o,c,di,dj] gy[n,o,i-di+1,j-dj+1]; if z given,
// the result is masked by [z > 0] (gradient through the previous relu)
__global__ void k_conv3_bwd_x(int B, int Ci, int Co, int H, int W, const float* __restrict__ gy,
                              const float* __restrict__ w, const float* __restrict__ z, float* __restrict__ gx) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= int64_t(B) * Ci * H * W) return;
  const int j = int(idx % W), i = int((idx / W) % H), c = int((idx / (int64_t(W) * H)) % Ci);
  const int n = int(idx / (int64_t(W) * H * Ci));
  float s = 0.f;
  for (int o = 0; o < Co; ++o) {
    const float* go = gy + (int64_t(n) * Co + o) * H * W;
    const float* wo = w + (int64_t(o) * Ci + c) * 9;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = (i - di + 1 + H) % H;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) s += wo[di * 3 + dj] * go[ii * W + (j - dj + 1 + W) % W];
    }
  }
  gx[idx] = (z == nullptr || z[idx] > 0.f) ? s : 0.f;
}

// gW[o,c,di,dj] = sum_{n,i,j} gy[n,o,i,j] x[n,c,i+di-1,j+dj-1], gb[o] = sum gy[n,o]
__global__ void k_conv3_bwd_w(int B, int Ci, int Co, int H, int W, const float* __restrict__ gy,
                              const float* __restrict__ x, float* __restrict__ gw, float* __restrict__ gb) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int nw = Co * Ci * 9;
  if (idx < nw) {
    const int t = idx % 9, c = (idx / 9) % Ci, o = idx / (9 * Ci);
    const int di = t / 3, dj = t % 3;
    float s = 0.f;
    for (int n = 0; n < B; ++n) {
      const float* go = gy + (int64_t(n) * Co + o) * H * W;
      const float* xc = x + (int64_t(n) * Ci + c) * H * W;
      for (int i = 0; i < H; ++i) {
        const int ii = (i + di - 1 + H) % H;
        for (int j = 0; j < W; ++j) s += go[i * W + j] * xc[ii * W + (j + dj - 1 + W) % W];
      }
    }
    gw[idx] = s;
  } else if (idx < nw + Co) {
    const int o = idx - nw;
    float s = 0.f;
    for (int n = 0; n < B; ++n)
      for (int p = 0; p < H * W; ++p) s += gy[(int64_t(n) * Co + o) * H * W + p];
    gb[o] = s;
  }
}

__global__ void k_adam(int64_t P, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= P) return;
  const float mi = b1 * m[i] + (1.f - b1) * g[i];
  const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

struct tdslda_nn {
  int H = 0, W = 0, C = 0, Bmax = 0;
  int64_t P = 0;
  int64_t off[10] = {0};
  int64_t t = 0;
  std::vector<void*> owned;
  float *th = nullptr, *gr = nullptr, *m = nullptr, *v = nullptr;
  float *x = nullptr, *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *z3 = nullptr, *h3 = nullptr;
  float *maps = nullptr, *g = nullptr, *mu = nullptr, *Y = nullptr, *ymu = nullptr;
  float *gmaps = nullptr, *gmu = nullptr, *ga = nullptr, *gb_ = nullptr, *loss = nullptr;
  std::string err;

  float* alloc(int64_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(float) * size_t(n)) != hipSuccess) {
      (void)hipGetLastError();
      throw NnFail{TDSLDA_ENOMEM, "hipMalloc failed (network buffers)"};
    }
    owned.push_back(p);
    return (float*)p;
  }
  ~tdslda_nn() {
    (void)hipDeviceSynchronize();
    for (void* p : owned) (void)hipFree(p);
  }
  float* par(int k) const { return th + off[k]; }
  float* grd(int k) const { return gr + off[k]; }

  void forward(int B) {
    const int HW = H * W;
    const int64_t act = int64_t(B) * C * HW;
    hipLaunchKernelGGL(k_conv3_fwd, dim3(nblk(act)), dim3(256), 0, 0, B, 1, C, H, W, x, par(0), par(1), z1, h1);
    hipLaunchKernelGGL(k_conv3_fwd, dim3(nblk(act)), dim3(256), 0, 0, B, C, C, H, W, h1, par(2), par(3), z2, h2);
    hipLaunchKernelGGL(k_conv3_fwd, dim3(nblk(act)), dim3(256), 0, 0, B, C, C, H, W, h2, par(4), par(5), z3, h3);
    hipLaunchKernelGGL(k_head_fwd, dim3(nblk(int64_t(B) * 2 * HW)), dim3(256), 0, 0, B, C, HW, h3, par(6), par(7),
                       maps);
    hipLaunchKernelGGL(k_gap, dim3(nblk(B * C)), dim3(256), 0, 0, B, C, HW, h3, g);
    hipLaunchKernelGGL(k_mu, dim3(nblk(B)), dim3(256), 0, 0, B, C, g, par(8), par(9), mu);
    NNCHK(hipGetLastError());
  }
  void backward(int B, float lam) {
    const int HW = H * W;
    const int64_t act = int64_t(B) * C * HW;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, 0, B, HW, maps, Y, mu, ymu, lam, gmaps, gmu, loss);
    hipLaunchKernelGGL(k_head_bwd_w, dim3(nblk(3 * C + 3)), dim3(256), 0, 0, B, C, HW, gmaps, h3, g, gmu, grd(6),
                       grd(7), grd(8), grd(9));
    hipLaunchKernelGGL(k_head_bwd_x, dim3(nblk(act)), dim3(256), 0, 0, B, C, HW, gmaps, gmu, par(6), par(8), z3, ga);
    // layer 3: gz3 in ga
    hipLaunchKernelGGL(k_conv3_bwd_w, dim3(nblk(C * C * 9 + C)), dim3(256), 0, 0, B, C, C, H, W, ga, h2, grd(4),
                       grd(5));
    hipLaunchKernelGGL(k_conv3_bwd_x, dim3(nblk(act)), dim3(256), 0, 0, B, C, C, H, W, ga, par(4), z2, gb_);
    // layer 2: gz2 in gb_
    hipLaunchKernelGGL(k_conv3_bwd_w, dim3(nblk(C * C * 9 + C)), dim3(256), 0, 0, B, C, C, H, W, gb_, h1, grd(2),
                       grd(3));
    hipLaunchKernelGGL(k_conv3_bwd_x, dim3(nblk(act)), dim3(256), 0, 0, B, C, C, H, W, gb_, par(2), z1, ga);
    // layer 1: gz1 in ga
    hipLaunchKernelGGL(k_conv3_bwd_w, dim3(nblk(C * 9 + C)), dim3(256), 0, 0, B, 1, C, H, W, ga, x, grd(0), grd(1));
    NNCHK(hipGetLastError());
  }
  void upload(const float* xh, int B) { NNCHK(hipMemcpy(x, xh, sizeof(float) * size_t(B) * H * W, hipMemcpyHostToDevice)); }
};

namespace {
template <class F>
tdslda_status nn_guard(tdslda_nn* n, F&& f) {
  try {
    f();
    return TDSLDA_OK;
  } catch (const NnFail& e) {
    if (n) n->err = e.msg;
    std::fprintf(stderr, "tdslda_nn: %s\n", e.msg.c_str());
    return e.st;
  } catch (...) {
    return TDSLDA_EDEVICE;
  }
}
}  // namespace

extern "C" {

int64_t tdslda_nn_nparams(int C) {
  if (C <= 0) return -1;
  return int64_t(C) * 9 + C + 2 * (int64_t(C) * C * 9 + C) + 2 * C + 2 + C + 1;
}

tdslda_status tdslda_nn_create(int H, int W, int C, int batch_max, const float* theta0, tdslda_nn** out) {
  if (!out || H <= 0 || W <= 0 || C <= 0 || batch_max <= 0 || !theta0) return TDSLDA_EINVAL;
  *out = nullptr;
  tdslda_nn* n = new (std::nothrow) tdslda_nn();
  if (!n) return TDSLDA_ENOMEM;
  const tdslda_status st = nn_guard(n, [&] {
    n->H = H;
    n->W = W;
    n->C = C;
    n->Bmax = batch_max;
    n->P = tdslda_nn_nparams(C);
    const int64_t sz[10] = {int64_t(C) * 9, C, int64_t(C) * C * 9, C, int64_t(C) * C * 9, C, 2 * int64_t(C), 2, C, 1};
    int64_t o = 0;
    for (int k = 0; k < 10; ++k) {
      n->off[k] = o;
      o += sz[k];
    }
    n->th = n->alloc(n->P);
    n->gr = n->alloc(n->P);
    n->m = n->alloc(n->P);
    n->v = n->alloc(n->P);
    NNCHK(hipMemcpy(n->th, theta0, sizeof(float) * n->P, hipMemcpyHostToDevice));
    NNCHK(hipMemset(n->m, 0, sizeof(float) * n->P));
    NNCHK(hipMemset(n->v, 0, sizeof(float) * n->P));
    const int64_t HW = int64_t(H) * W, act = int64_t(batch_max) * C * HW;
    n->x = n->alloc(batch_max * HW);
    for (float** p : {&n->z1, &n->h1, &n->z2, &n->h2, &n->z3, &n->h3, &n->ga, &n->gb_}) *p = n->alloc(act);
    n->maps = n->alloc(int64_t(batch_max) * 2 * HW);
    n->Y = n->alloc(int64_t(batch_max) * 2 * HW);
    n->gmaps = n->alloc(int64_t(batch_max) * 2 * HW);
    n->g = n->alloc(int64_t(batch_max) * C);
    n->mu = n->alloc(batch_max);
    n->ymu = n->alloc(batch_max);
    n->gmu = n->alloc(batch_max);
    n->loss = n->alloc(1);
  });
  if (st != TDSLDA_OK) {
    delete n;
    return st;
  }
  *out = n;
  return TDSLDA_OK;
}

tdslda_status tdslda_nn_destroy(tdslda_nn* n) {
  if (!n) return TDSLDA_EINVAL;
  delete n;
  return TDSLDA_OK;
}

tdslda_status tdslda_nn_params(tdslda_nn* n, float* theta_out, int64_t* count) {
  if (!n) return TDSLDA_EINVAL;
  return nn_guard(n, [&] {
    if (count) *count = n->P;
    if (theta_out) NNCHK(hipMemcpy(theta_out, n->th, sizeof(float) * n->P, hipMemcpyDeviceToHost));
  });
}

tdslda_status tdslda_nn_set_params(tdslda_nn* n, const float* theta) {
  if (!n || !theta) return TDSLDA_EINVAL;
  return nn_guard(n, [&] {
    NNCHK(hipMemcpy(n->th, theta, sizeof(float) * n->P, hipMemcpyHostToDevice));
    NNCHK(hipMemset(n->m, 0, sizeof(float) * n->P));
    NNCHK(hipMemset(n->v, 0, sizeof(float) * n->P));
    n->t = 0;
  });
}

tdslda_status tdslda_nn_forward(tdslda_nn* n, int B, const float* x, float* maps, float* mu) {
  if (!n || !x || B <= 0 || B > (n ? n->Bmax : 0)) return TDSLDA_EINVAL;
  return nn_guard(n, [&] {
    n->upload(x, B);
    n->forward(B);
    const size_t HW = size_t(n->H) * n->W;
    if (maps) NNCHK(hipMemcpy(maps, n->maps, sizeof(float) * B * 2 * HW, hipMemcpyDeviceToHost));
    if (mu) NNCHK(hipMemcpy(mu, n->mu, sizeof(float) * B, hipMemcpyDeviceToHost));
  });
}

tdslda_status tdslda_nn_loss_grad(tdslda_nn* n, int B, const float* x, const float* Y, const float* ymu,
                                  float lam_mu, float* loss, float* grad) {
  if (!n || !x || !Y || !ymu || B <= 0 || B > (n ? n->Bmax : 0)) return TDSLDA_EINVAL;
  return nn_guard(n, [&] {
    const size_t HW = size_t(n->H) * n->W;
    n->upload(x, B);
    NNCHK(hipMemcpy(n->Y, Y, sizeof(float) * B * 2 * HW, hipMemcpyHostToDevice));
    NNCHK(hipMemcpy(n->ymu, ymu, sizeof(float) * B, hipMemcpyHostToDevice));
    n->forward(B);
    n->backward(B, lam_mu);
    if (loss) NNCHK(hipMemcpy(loss, n->loss, sizeof(float), hipMemcpyDeviceToHost));
    if (grad) NNCHK(hipMemcpy(grad, n->gr, sizeof(float) * n->P, hipMemcpyDeviceToHost));
  });
}

tdslda_status tdslda_nn_train_step(tdslda_nn* n, int B, const float* x, const float* Y, const float* ymu,
                                   float lam_mu, float lr, float* loss) {
  const tdslda_status st = tdslda_nn_loss_grad(n, B, x, Y, ymu, lam_mu, loss, nullptr);
  if (st != TDSLDA_OK) return st;
  return nn_guard(n, [&] {
    n->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(n->t)), c2 = 1.f - std::pow(b2, float(n->t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->P)), dim3(256), 0, 0, n->P, n->th, n->gr, n->m, n->v, lr, b1, b2, 1e-8f,
                       c1, c2);
    NNCHK(hipGetLastError());
    NNCHK(hipDeviceSynchronize());
  });
}

}  // extern "C"
