// Device kernels of the full-3D TDSLDA path (gfx950).
//
// States are stored [n][u|v][ixyz] as interleaved complex of R (double or
// float); ixyz = (ix*NY + iy)*NZ + iz.  The Laplacian is split by axis
// (the Kronecker sum of the D^(2) matrices of Eq. D2, each applied as an
// FFT along that axis):
//   - lap1 (x-lines): one thread owns one x-line of one state, FFTs it in
//     registers and writes D2x phi to the intermediate buffer T;
//   - dens / lap2 (x-slabs): a workgroup owns SX consecutive x-slabs of a
//     state; the (y,z) part of the Laplacian is a 2D spectral transform in
//     LDS (z-lines, then y-lines, then z-lines back), one thread per line.
// Everything reduced over sites or states is accumulated in FP64 in a fixed
// order (no floating-point atomics), so results are reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include "bufio.h"
#include "fft.h"

namespace tdslda {

constexpr int kWave = 64;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over the block; every thread gets the result.  scratch: >= nwaves doubles.
template <int TB>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  constexpr int NW = (TB + kWave - 1) / kWave;
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) scratch[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += scratch[i];
  return s;
}

template <typename R>
__device__ __forceinline__ double norm2(cpx<R> a) {
  return double(a.x) * double(a.x) + double(a.y) * double(a.y);
}

// ---------------------------------------------------------------------------
// compile-time tiling of the slab kernels
// Tiling knobs (compile-time): lines per slab workgroup target and the
// largest sites-per-thread count for which the fused pass keeps its sites
// of phi in registers instead of re-reading them.  Defaults: 32 lines (one
// x-slab per workgroup at 32^3: 35 KB of LDS and 104 VGPRs with the
// lane-pair lines, four workgroups per CU; two x-slabs took 2% more per
// 32^3 FP64 step), no stash (the stash gains nothing at 32^3 FP64).
#ifndef TDSLDA_SLAB_LINES
#define TDSLDA_SLAB_LINES 32
#endif
#ifndef TDSLDA_STASH_MAXP
#define TDSLDA_STASH_MAXP 0
#endif

template <int NX, int NY, int NZ>
struct SlabCfg {
  static constexpr int NXv = NX, NYv = NY, NZv = NZ;
  static constexpr int NMAX = NY > NZ ? NY : NZ;
  static constexpr int sx_target() {
    int t = TDSLDA_SLAB_LINES / NMAX;
    if (t < 1) t = 1;
    while (NX % t) --t;
    return t;
  }
  static constexpr int SX = sx_target();          // x-slabs per workgroup
  static constexpr int NYZ = NY * NZ;
  static constexpr int SS = SX * NYZ;             // sites per workgroup
  // line phases: a lane pair per line (the lane-pair DFT of fft.h)
  static constexpr int TASKS = ((4 * SX * NMAX + kWave - 1) / kWave) * kWave;  // line lanes
  static constexpr int TB = TASKS > 256 ? TASKS : 256;  // threads (line phases use the first TASKS)
  static constexpr int P = (SS + TB - 1) / TB;    // sites per thread
  static constexpr int NGX = NX / SX;             // workgroups per state
  static constexpr int PADZ = NZ + 2;             // LDS row pitch (bank spread of the lane pairs)
  static constexpr int LDS_ELEMS = 2 * SX * NY * PADZ;
  __device__ static int lds_index(int comp, int p) {
    int sx = p / NYZ, rem = p - sx * NYZ, y = rem / NZ, z = rem - y * NZ;
    return ((comp * SX + sx) * NY + y) * PADZ + z;
  }
};

// in-LDS line transforms of the slab block -----------------------------------
// Each line is held by a lane pair: lane parity b owns the samples 2j + b
// of the line (the LDS row positions 2j + b), in place.  After the forward
// transform, row position q = 2p + b holds the frequency of position p of
// lane b (pair_wavenum_at<N>(q) gives its signed wave number).
//
// z-line transform of every (comp, sx, y) line: SIGN < 0 forward (natural z
// in), SIGN > 0 inverse (back to natural z).
template <class CFG, int SIGN, typename R>
__device__ __forceinline__ void lds_zlines(cpx<R>* lds) {
  constexpr int NZ = CFG::NZv, NY = CFG::NYv, HZ = NZ / 2;
  constexpr int lines = 2 * CFG::SX * NY;
  const int t = threadIdx.x >> 1;
  const bool odd = threadIdx.x & 1;
  if (t < lines) {  // both lanes of a pair
    cpx<R>* base = lds + t * CFG::PADZ + (odd ? 1 : 0);  // (comp*SX + sx)*NY + y == t
    cpx<R> a[HZ];
#pragma unroll
    for (int j = 0; j < HZ; ++j) a[j] = base[2 * j];
    if constexpr (SIGN < 0) {
      fwd_pair<NZ>(a, odd);
    } else {
      inv_pair<NZ>(a, odd);
    }
#pragma unroll
    for (int j = 0; j < HZ; ++j) base[2 * j] = a[j];
  }
}

// the y-line of a lane pair after the z-lines' forward transform: its
// component, slab plane and k_z row position
template <class CFG>
struct YLine {
  int comp, sx, kz;
  bool odd, live;
  __device__ YLine() {
    constexpr int NZ = CFG::NZv;
    const int t = threadIdx.x >> 1;
    odd = threadIdx.x & 1;
    live = t < 2 * CFG::SX * NZ;  // both lanes of a pair
    comp = t / (CFG::SX * NZ);
    const int rem = t - comp * CFG::SX * NZ;
    sx = rem / NZ;
    kz = rem - sx * NZ;
  }
  template <typename R>
  __device__ cpx<R>* base(cpx<R>* lds) const {
    return lds + ((comp * CFG::SX + sx) * CFG::NYv + (odd ? 1 : 0)) * CFG::PADZ + kz;
  }
};

// (y,z) kinetic part of <H> from a slab whose z-lines were forward
// transformed in place: each y-line pair transforms its column forward and
// returns (+1/2 for u, -1/2 for v) sum_k (ky^2 + kz^2) |phi_k|^2 dV / (NY NZ)
// over its half of the column (Parseval; zero for threads without a line).
template <class CFG, typename R>
__device__ __forceinline__ double lds_yz_kinetic(const cpx<R>* lds, double cy2, double cz2, double dV) {
  constexpr int NY = CFG::NYv, NZ = CFG::NZv, HY = NY / 2;
  const YLine<CFG> yl;
  if (!yl.live) return 0.0;
  const cpx<R>* base = yl.base(const_cast<cpx<R>*>(lds));
  cpx<R> a[HY];
#pragma unroll
  for (int j = 0; j < HY; ++j) a[j] = base[2 * j * CFG::PADZ];
  fwd_pair<NY>(a, yl.odd);
  const int mz = pair_wavenum_at<NZ>(yl.kz);
  const double ez = cz2 * double(mz * mz);
  double acc = 0.0;
  sfor<0, HY>::run([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const int my = pair_wavenum<NY, j>(yl.odd);
    acc += (cy2 * double(my * my) + ez) * norm2(a[j]);
  });
  return (yl.comp == 0 ? 0.5 : -0.5) * acc * dV / double(CFG::NYZ);
}

// ---------------------------------------------------------------------------
// Per-state scalars: norm^2 partials (one slot per slab group) and <H>_n
// partials (slab-group slots from dens, column-block slots from lap1).
struct StateScalars {
  double* nrm_part;  // [n][nrm_stride]
  int nrm_stride;
  double* h_part;    // [n][h_stride]
  int h_stride;
  int h_lap1_off;    // first lap1 slot
  double* scale;     // [n] 1/sqrt(norm^2)
  double* hshift;    // [n] <H>_n
};

// ---------------------------------------------------------------------------
// dens: densities rho, nu of the normalised states (Eqs. nab3D and the
// anomalous density of the spin-symmetric case) as per-state-group partial
// sums, plus the y,z kinetic part of <H>_n of the stored (unscaled) state.
//   grid = (NGX, number of state groups), block = CFG::TB
//   dens_part layout [group][3][M] (rho, Re nu, Im nu)
template <typename R, int NX, int NY, int NZ, int G>
__global__ __launch_bounds__((SlabCfg<NX, NY, NZ>::TB)) void k_dens(
    const cpx<R>* __restrict__ X, int64_t nstates, const double* __restrict__ wu,
    const double* __restrict__ wv, StateScalars sc, double* __restrict__ dens_part,
    double cy2, double cz2, double dV) {
  using CFG = SlabCfg<NX, NY, NZ>;
  constexpr int TB = CFG::TB, P = CFG::P, SS = CFG::SS, NYZ = CFG::NYZ;
  constexpr int M = NX * NYZ;
  constexpr int NW = TB / kWave;
  __shared__ cpx<R> lds[CFG::LDS_ELEMS];
  __shared__ double kin[G][NW];
  const int g = blockIdx.x, sg = blockIdx.y, tid = threadIdx.x;
  const int64_t site0 = int64_t(g) * SS;
  double ar[P], anr[P], ani[P];
#pragma unroll
  for (int i = 0; i < P; ++i) ar[i] = anr[i] = ani[i] = 0.0;

  const int64_t nbeg = int64_t(sg) * G;
  for (int ls = 0; ls < G; ++ls) {
    const int64_t n = nbeg + ls;
    const bool live = n < nstates;  // uniform over the block
    if (live) {
      constexpr int ES = sizeof(cpx<R>);
      const double s = sc.scale[n], fu = wu[n], fv = wv[n];
      const bi32x4 rX = make_rsrc(X + n * 2 * M, 2 * M * ES);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int p = tid + i * TB;
        if (p < SS) {
          const int so = int(site0 + i * TB) * ES;
          const cpx<R> xu = bload<R>(rX, tid * ES, so), xv = bload<R>(rX, tid * ES, so + M * ES);
          const cpx<R> u = R(s) * xu, v = R(s) * xv;
          const double ur = u.x, ui = u.y, vr = v.x, vi = v.y;
          ar[i] += fv * (vr * vr + vi * vi) + fu * (ur * ur + ui * ui);
          const double dw = fv - fu;  // u v^*
          anr[i] += dw * (ur * vr + ui * vi);
          ani[i] += dw * (ui * vr - ur * vi);
          // the kinetic partial is taken on the stored (unscaled) values;
          // the finalisation multiplies it by scale^2
          lds[CFG::lds_index(0, p)] = xu;
          lds[CFG::lds_index(1, p)] = xv;
        }
      }
    }
    __syncthreads();
    if (live) lds_zlines<CFG, -1>(lds);
    __syncthreads();
    double kv = 0.0;
    if (live) kv = lds_yz_kinetic<CFG, R>(lds, cy2, cz2, dV);
    kv = wave_sum(kv);
    if (tid % kWave == 0) kin[ls][tid / kWave] = kv;
    __syncthreads();
  }
  // density partials of this state group
  double* out = dens_part + int64_t(sg) * 3 * M + site0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int p = tid + i * TB;
    if (p < SS) {
      out[p] = ar[i];
      out[M + p] = anr[i];
      out[2 * M + p] = ani[i];
    }
  }
  if (tid < G) {
    const int64_t n = nbeg + tid;
    if (n < nstates) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += kin[tid][w];
      sc.h_part[n * sc.h_stride + g] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// dens_sum: the density partials only (rho, nu of the normalised states), for
// states whose (y,z) kinetic partial was already produced by the kernel that
// wrote them.  Site-parallel, no LDS: a thread owns DS_P sites (stride TB) and
// walks the DG states of its group, so every load is a coalesced row.
//   grid = (ceil(M / (TB DS_P)), ceil(nstates / DG)), block = TB
//   dens_part layout [group][3][M]
constexpr int DS_TB = 256, DS_P = 2;
// NC: components per group in the partial layout (3; more when further
// components, written by another pass, follow).  SPIN: the spin-resolved
// densities of both branches (Eqs. na3D-jb3D): rho_a = sum f_u |u|^2,
// rho_b = sum f_v |v|^2 and nu = 1/2 sum (f_v - f_u) u v^*, in components
// 0 .. 3 (rho_a, rho_b, Re nu, Im nu).
template <typename R, int DG, int PS = DS_P, int NC = 3, bool SPIN = false>
__global__ __launch_bounds__(DS_TB) void k_dens_sum(
    const cpx<R>* __restrict__ X, int64_t nstates, int64_t M, const double* __restrict__ wu,
    const double* __restrict__ wv, const double* __restrict__ scale, double* __restrict__ dens_part) {
  const int tid = threadIdx.x;
  const int64_t site0 = int64_t(blockIdx.x) * (DS_TB * PS) + tid;
  const int64_t nbeg = int64_t(blockIdx.y) * DG;
  const int nloc = int(nstates - nbeg < DG ? nstates - nbeg : DG);
  double ar[PS], ab[SPIN ? PS : 1], anr[PS], ani[PS];
#pragma unroll
  for (int i = 0; i < PS; ++i) {
    ar[i] = anr[i] = ani[i] = 0.0;
    if constexpr (SPIN) ab[i] = 0.0;
  }
  const cpx<R>* xb = X + nbeg * 2 * M;
#pragma unroll 4
  for (int ls = 0; ls < nloc; ++ls) {
    const double s = scale[nbeg + ls], fu = wu[nbeg + ls], fv = wv[nbeg + ls];
    const double s2 = s * s, cu = fu * s2, cv = fv * s2, cw = (SPIN ? 0.5 : 1.0) * (fv - fu) * s2;
    const cpx<R>* xs = xb + int64_t(ls) * 2 * M;
#pragma unroll
    for (int i = 0; i < PS; ++i) {
      const int64_t r = site0 + i * DS_TB;
      if (r < M) {
        const cpx<R> u = ld_stream(xs + r), v = ld_stream(xs + M + r);
        const double ur = u.x, ui = u.y, vr = v.x, vi = v.y;
        if constexpr (SPIN) {
          ar[i] += cu * (ur * ur + ui * ui);
          ab[i] += cv * (vr * vr + vi * vi);
        } else {
          ar[i] += cv * (vr * vr + vi * vi) + cu * (ur * ur + ui * ui);
        }
        anr[i] += cw * (ur * vr + ui * vi);  // u v^*
        ani[i] += cw * (ui * vr - ur * vi);
      }
    }
  }
  double* out = dens_part + int64_t(blockIdx.y) * NC * M;
  constexpr int ON = SPIN ? 2 : 1;  // first nu component
#pragma unroll
  for (int i = 0; i < PS; ++i) {
    const int64_t r = site0 + i * DS_TB;
    if (r < M) {
      out[r] = ar[i];
      if constexpr (SPIN) out[M + r] = ab[i];
      out[ON * M + r] = anr[i];
      out[(ON + 1) * M + r] = ani[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Functional parameters used by the pointwise potential kernel.
struct FunParams {
  int kind;            // 1 SLDA, 2 BdG
  double B, C, inv_g;  // constants
  double mu;
  double ainv;         // 1 in 3D, 1/(L_x L_y) in quasi-1D
  const double* dext;  // external pairing potential [M][2] (added to Delta in H)
};

// reduce_pot: sum the state-group partials (fixed order) and build the
// potentials pointwise: Delta = -g_eff nu with 1/g_eff = rho_+^(1/3)/C -
// Lambda_c (SLDA) or 1/(4 pi a_s) - Lambda_c (BdG), U = B eF(rho_+) -
// |Delta|^2 / (3 C rho_+^(2/3)) (SLDA, A=1) or 0 (BdG).  The off-diagonal
// field of H is Delta + Delta_ext (Eq. HpsiEpsi).
template <typename R>
__device__ __forceinline__ void pot_from_sums(int64_t r, double sr, double snr, double sni, const FunParams& fp,
                                              const double* __restrict__ lam, const double* __restrict__ vext,
                                              double* __restrict__ rho, double* __restrict__ nu,
                                              double* __restrict__ U, double* __restrict__ delta,
                                              R* __restrict__ hA, cpx<R>* __restrict__ hD, int update_fields) {
  sr *= fp.ainv;
  snr *= fp.ainv;
  sni *= fp.ainv;
  rho[r] = sr;
  nu[2 * r] = snr;
  nu[2 * r + 1] = sni;
  if (!update_fields) return;
  const double rp = fmax(2.0 * sr, 1e-14);
  double ig;
  if (fp.kind == 1) {
    ig = cbrt(rp) / fp.C - lam[r];
  } else {
    ig = fp.inv_g - lam[r];
  }
  const double gg = 1.0 / ig;
  const double dr = -gg * snr, di = -gg * sni;
  double u = 0.0;
  if (fp.kind == 1) {
    const double ef = 0.5 * pow(3.0 * kPi * kPi * (2.0 * sr), 2.0 / 3.0);
    const double c23 = cbrt(rp);
    u = fp.B * ef - (dr * dr + di * di) / (3.0 * fp.C * c23 * c23);
  }
  U[r] = u;
  delta[2 * r] = dr;
  delta[2 * r + 1] = di;
  hA[r] = R(u + vext[r] - fp.mu);
  hD[r] = cpx<R>{R(dr + fp.dext[2 * r]), R(di + fp.dext[2 * r + 1])};
}

// one thread per site, groups summed in order
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_pot(
    const double* __restrict__ dens_part, int ngroups, int64_t M, FunParams fp,
    const double* __restrict__ lam, const double* __restrict__ vext, double* __restrict__ rho,
    double* __restrict__ nu, double* __restrict__ U, double* __restrict__ delta,
    R* __restrict__ hA, cpx<R>* __restrict__ hD, int update_fields) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double sr = 0.0, snr = 0.0, sni = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const double* p = dens_part + int64_t(g) * 3 * M;
    sr += p[r];
    snr += p[M + r];
    sni += p[2 * M + r];
  }
  pot_from_sums<R>(r, sr, snr, sni, fp, lam, vext, rho, nu, U, delta, hA, hD, update_fields);
}

// one workgroup per site (few sites, many groups): thread t sums groups
// t, t + 256, ... in order, then a fixed-order tree over the threads
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_pot_wide(
    const double* __restrict__ dens_part, int ngroups, int64_t M, FunParams fp,
    const double* __restrict__ lam, const double* __restrict__ vext, double* __restrict__ rho,
    double* __restrict__ nu, double* __restrict__ U, double* __restrict__ delta,
    R* __restrict__ hA, cpx<R>* __restrict__ hD, int update_fields) {
  __shared__ double t3[3][256];
  const int64_t r = blockIdx.x;
  const int t = threadIdx.x;
  double sr = 0.0, snr = 0.0, sni = 0.0;
  for (int g = t; g < ngroups; g += 256) {
    const double* p = dens_part + int64_t(g) * 3 * M;
    sr += p[r];
    snr += p[M + r];
    sni += p[2 * M + r];
  }
  t3[0][t] = sr;
  t3[1][t] = snr;
  t3[2][t] = sni;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) {
      t3[0][t] += t3[0][t + k];
      t3[1][t] += t3[1][t + k];
      t3[2][t] += t3[2][t + k];
    }
    __syncthreads();
  }
  if (t == 0) pot_from_sums<R>(r, t3[0][0], t3[1][0], t3[2][0], fp, lam, vext, rho, nu, U, delta, hA, hD,
                               update_fields);
}

// Frozen fields (linear mode): hA, hD from given U, Delta (hD = Delta +
// Delta_ext).
template <typename R>
__global__ void k_set_fields(int64_t M, const double* __restrict__ U, const double* __restrict__ delta,
                             const double* __restrict__ vext, const double* __restrict__ dext, double mu,
                             R* __restrict__ hA, cpx<R>* __restrict__ hD) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  hA[r] = R(U[r] + vext[r] - mu);
  hD[r] = cpx<R>{R(delta[2 * r] + dext[2 * r]), R(delta[2 * r + 1] + dext[2 * r + 1])};
}

// ---------------------------------------------------------------------------
// lap1: T = D2x phi for every state (x-lines, one thread per (y,z) column),
// plus the x kinetic part and the potential part of <H>_n:
//   1/2 int (|d_x u|^2 - |d_x v|^2) + int [A (|u|^2 - |v|^2) + 2 Re(u^* Delta v)]
//   grid = (ceil(NYZ/TB1), nstates), block = TB1
template <typename R, int NX, int NYZ, int TB1>
__global__ __launch_bounds__(TB1) void k_lap1(
    const cpx<R>* __restrict__ X, const double* __restrict__ scale, cpx<R>* __restrict__ T,
    const R* __restrict__ hA, const cpx<R>* __restrict__ hD, double* __restrict__ h_part, int h_stride,
    int h_off, double kx2, double dV) {
  __shared__ double red[TB1 / kWave];
  constexpr int64_t M = int64_t(NX) * NYZ;
  const int q = blockIdx.x * TB1 + threadIdx.x;
  const int64_t n = blockIdx.y;
  const bool act = q < NYZ;
  const R s = scale ? R(scale[n]) : R(1);
  // buffer resources over this state; rows addressed by scalar offsets,
  // the column by the lane offset
  constexpr int ES = sizeof(cpx<R>), RS = sizeof(R);
  const bi32x4 rX = make_rsrc(X + n * 2 * M, 2 * M * ES);
  const bi32x4 rT = make_rsrc(T + n * 2 * M, 2 * M * ES);
  const bi32x4 rA = make_rsrc(hA, M * RS);
  const bi32x4 rD = make_rsrc(hD, M * ES);
  const int vq = q * ES, vqa = q * RS;
  constexpr bool SPLIT_POT = sizeof(R) == 8;
  double hsum = 0.0;
  if (act) {
    cpx<R> a[NX];
    double kin = 0.0, pot = 0.0;
#pragma unroll 1
    for (int comp = 0; comp < 2; ++comp) {
      const double sg = comp ? -1.0 : 1.0;
      // lines that the potential part reads again stay cached; the rest stream
      if (h_part && (comp == 0 || !SPLIT_POT)) {
#pragma unroll
        for (int x = 0; x < NX; ++x) a[x] = s * bload<R>(rX, vq, int(comp * M + x * NYZ) * ES);
      } else {
#pragma unroll
        for (int x = 0; x < NX; ++x) a[x] = s * bload_nt<R>(rX, vq, int(comp * M + x * NYZ) * ES);
      }
      // potential part A (|u|^2 - |v|^2) + 2 Re(u^* Delta v), only when <H>_n
      // is wanted.  FP64: A |u|^2 in the u pass, -A |v|^2 and the cross term
      // in the v pass, which re-reads u (keeping the u line for the v pass
      // costs more in occupancy than the half re-read).  FP32: after both
      // passes, re-reading u and v (fewer live registers, measured faster).
      if (SPLIT_POT && h_part) {
#pragma unroll
        for (int x = 0; x < NX; ++x) {
          const double fa = double(bload_real<R>(rA, vqa, x * NYZ * RS));
          if (comp == 0) {
            pot += fa * norm2(a[x]);
          } else {
            const cpx<R> u = s * bload_nt<R>(rX, vq, x * NYZ * ES);
            const cpx<R> dv = bload<R>(rD, vq, x * NYZ * ES) * a[x];
            pot += 2.0 * (double(u.x) * double(dv.x) + double(u.y) * double(dv.y)) - fa * norm2(a[x]);
          }
        }
      }
      // sum_x |d_x f|^2 = kx2 * ks / NX (Parseval)
      const double ks = second_derivative<NX>(a, R(kx2));
      kin += sg * kx2 * ks / double(NX);
#pragma unroll
      for (int x = 0; x < NX; ++x) bstore_nt<R>(a[x], rT, vq, int(comp * M + x * NYZ) * ES);
    }
    if (!SPLIT_POT && h_part) {
#pragma unroll 4
      for (int x = 0; x < NX; ++x) {
        const cpx<R> u = s * bload_nt<R>(rX, vq, x * NYZ * ES), v = s * bload_nt<R>(rX, vq, int(M + x * NYZ) * ES);
        const cpx<R> dv = bload<R>(rD, vq, x * NYZ * ES) * v;
        pot += double(bload_real<R>(rA, vqa, x * NYZ * RS)) * (norm2(u) - norm2(v));
        pot += 2.0 * (double(u.x) * double(dv.x) + double(u.y) * double(dv.y));
      }
    }
    hsum = (0.5 * kin + pot) * dV;
  }
  if (h_part) {
    double v = wave_sum(hsum);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < TB1 / kWave; ++w) t += red[w];
      h_part[n * h_stride + h_off + blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// lap2: (y,z) Laplacian in LDS + T -> H phi pointwise, then the mode's
// integrator arithmetic, all in one pass over the state.
enum Lap2Mode { L2_H = 0, L2_F = 1, L2_CORR = 2, L2_FULL = 3, L2_TAYLOR = 4 };

template <typename R>
struct Lap2Args {
  const cpx<R>* X;       // input states (also written in place by CORR / FULL)
  cpx<R>* Xout;          // CORR: phi_new, FULL: p (both == X)
  const cpx<R>* T;       // D2x of the (scaled) input
  const R* hA;           // U + V_ext - mu
  const cpx<R>* hD;      // Delta
  const double* scale;   // nullptr = 1
  const double* hshift;  // nullptr = 0
  cpx<R>* out;           // H / F / TAYLOR output, FULL: f_k
  cpx<R>* acc;           // TAYLOR accumulator
  const cpx<R>* hist[5]; // FULL: hist[1..D-1] = f_{k-1}, ...; CORR: hist[0] = c
  cpx<R>* cout;          // FULL: c output (in place over hist[D-1])
  double* nrm_part;      // partial norms of the written state (or nullptr)
  int nrm_stride;
  int np, nq;            // predictor / corrector lengths (AB_np, AM_nq)
  double b[5];           // dt * AB weights
  double a[5];           // dt * AM weights
  double tay_re, tay_im; // TAYLOR: coefficient of (H - h) psi
  int init_acc;
  double cy2, cz2;       // (2 pi / L_y)^2, (2 pi / L_z)^2
  double* h_part;        // CORR / FULL: (y,z) kinetic partial of the written state
  int h_stride;
  double dV;
};

// NP, NQ: predictor / corrector lengths of the integrator (FULL mode only),
// compile-time so that the history buffers are addressed without branches.
template <typename R, int NX, int NY, int NZ, int MODE, int NP = 4, int NQ = 5>
__global__ __launch_bounds__((SlabCfg<NX, NY, NZ>::TB)) void k_lap2(Lap2Args<R> A) {
  using CFG = SlabCfg<NX, NY, NZ>;
  constexpr int TB = CFG::TB, P = CFG::P, SS = CFG::SS;
  constexpr int M = NX * NY * NZ;
  __shared__ cpx<R> lds[CFG::LDS_ELEMS];
  __shared__ double red[TB / kWave];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t n = blockIdx.y;
  const int64_t site0 = int64_t(g) * SS;
  constexpr int ES = sizeof(cpx<R>), RS = sizeof(R);
  const R s = A.scale ? R(A.scale[n]) : R(1);
  const R h = A.hshift ? R(A.hshift[n]) : R(0);
  const int64_t so = n * 2 * M;
  const uint32_t SB = 2 * M * ES;
  const bi32x4 rX = make_rsrc(A.X + so, SB);
  const int vt = tid * ES;
  constexpr bool STASH = P <= TDSLDA_STASH_MAXP;
  cpx<R> xs[2][STASH ? P : 1];

#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int p = tid + i * TB;
    if (p < SS) {
      const int o = int(site0 + i * TB) * ES;
      const cpx<R> xu = s * bload<R>(rX, vt, o), xv = s * bload<R>(rX, vt, o + M * ES);
      lds[CFG::lds_index(0, p)] = xu;
      lds[CFG::lds_index(1, p)] = xv;
      if constexpr (STASH) {
        xs[0][i] = xu;
        xs[1][i] = xv;
      }
    }
  }
  __syncthreads();
  lds_zlines<CFG, -1>(lds);
  __syncthreads();
  {  // y-lines: forward, multiply by -(ky^2 + kz^2)/(NY NZ), inverse
    constexpr int HY = NY / 2;
    const YLine<CFG> yl;
    if (yl.live) {
      cpx<R>* lb = yl.base(lds);
      cpx<R> a[HY];
#pragma unroll
      for (int j = 0; j < HY; ++j) a[j] = lb[2 * j * CFG::PADZ];
      fwd_pair<NY>(a, yl.odd);
      const int mz = pair_wavenum_at<NZ>(yl.kz);
      const R ez = R(A.cz2 * double(mz * mz));
      const R nrm = R(-1.0 / double(NY * NZ));
      sfor<0, HY>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const int my = pair_wavenum<NY, j>(yl.odd);
        a[j] = (nrm * (R(A.cy2) * R(my * my) + ez)) * a[j];
      });
      inv_pair<NY>(a, yl.odd);
#pragma unroll
      for (int j = 0; j < HY; ++j) lb[2 * j * CFG::PADZ] = a[j];
    }
  }
  __syncthreads();
  lds_zlines<CFG, +1>(lds);
  __syncthreads();

  const bi32x4 rT = make_rsrc(A.T + so, SB);
  const bi32x4 rA = make_rsrc(A.hA, M * RS);
  const bi32x4 rD = make_rsrc(A.hD, M * ES);
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
    if (p < SS) {
      const int ou = int(site0 + i * TB) * ES, ov = ou + M * ES;
      const int oa = int(site0 + i * TB) * RS;
      const cpx<R> lu = lds[CFG::lds_index(0, p)] + bload_nt<R>(rT, vt, ou);
      const cpx<R> lv = lds[CFG::lds_index(1, p)] + bload_nt<R>(rT, vt, ov);
      const R fa = bload_real<R>(rA, tid * RS, oa);
      const cpx<R> D = bload<R>(rD, vt, ou);
      // phi is re-read unless the tiling keeps it (STASH): holding many sites
      // through the transforms halves the waves per SIMD
      cpx<R> u, v;
      if constexpr (STASH) {
        u = xs[0][i];
        v = xs[1][i];
      } else {
        u = s * bload_nt<R>(rX, vt, ou);
        v = s * bload_nt<R>(rX, vt, ov);
      }
      // H (u, v) = ( -1/2 lap u + A u + D v ,  D^* u + 1/2 lap v - A v )
      cpx<R> Hu = R(-0.5) * lu + fa * u + D * v;
      cpx<R> Hv = conj(D) * u + R(0.5) * lv - fa * v;
      if constexpr (MODE == L2_H) {
        bstore_nt<R>(Hu, rO, vt, ou);
        bstore_nt<R>(Hv, rO, vt, ov);
      } else {
        // f = -i (H - h) phi
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
            // the written state replaces this thread's own LDS sites
            lds[CFG::lds_index(0, p)] = nu_;
            lds[CFG::lds_index(1, p)] = nv_;
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
            lds[CFG::lds_index(0, p)] = pu;
            lds[CFG::lds_index(1, p)] = pv;
          }
        }
      }
    }
  }
  if constexpr (MODE == L2_CORR || MODE == L2_FULL) {
    // (y,z) kinetic partial of the state just written (unscaled), so that
    // the next evaluation's density pass needs no transform
    __syncthreads();
    lds_zlines<CFG, -1>(lds);
    __syncthreads();
    const double kv = lds_yz_kinetic<CFG, R>(lds, A.cy2, A.cz2, A.dV);
    const double t = block_sum<TB>(kv, red);
    if (tid == 0) A.h_part[n * A.h_stride + g] = t;
  }
  if (A.nrm_part) {
    const double t = block_sum<TB>(nacc, red);
    if (tid == 0) A.nrm_part[n * A.nrm_stride + g] = t;
  }
}

// ---------------------------------------------------------------------------
// Pointwise kernels over the slab-group tiling (same norm-partial slots).
enum PwMode { PW_NORM = 0, PW_PRED = 1, PW_SCALE = 2 };

template <typename R>
struct PwArgs {
  cpx<R>* X;
  const double* scale;
  const cpx<R>* hist[5];  // PRED: f_{k-1}, ..., f_{k-D}
  cpx<R>* cout;           // PRED: c (in place over hist[D-1])
  double* nrm_part;
  int nrm_stride;
  int np, nq;
  double b[5], a[5];
  cpx<double>* out64;     // SCALE: FP64 copy of the normalised state
  int64_t nst;            // states (grid rows stride over them)
};

// grid rows of a per-state launch: states beyond it are strided over
inline unsigned state_rows(int64_t nst) { return unsigned(nst < 65535 ? nst : 65535); }

template <typename R, int NX, int NY, int NZ, int MODE, int NP = 4, int NQ = 5>
__global__ __launch_bounds__((SlabCfg<NX, NY, NZ>::TB)) void k_pointwise(PwArgs<R> A) {
  using CFG = SlabCfg<NX, NY, NZ>;
  constexpr int TB = CFG::TB, P = CFG::P, SS = CFG::SS;
  constexpr int M = NX * NY * NZ;
  __shared__ double red[TB / kWave];
  const int g = blockIdx.x, tid = threadIdx.x;
  for (int64_t n = blockIdx.y; n < A.nst; n += gridDim.y) {
  constexpr int ES = sizeof(cpx<R>);
  const int64_t so = n * 2 * M;
  const uint32_t SB = 2 * M * ES;
  const bi32x4 rX = make_rsrc(A.X + so, SB);
  constexpr int HD = (NP > NQ - 1) ? NP : NQ - 1;
  bi32x4 rH[HD] = {}, rC{};
  if constexpr (MODE == PW_PRED) {
    rC = make_rsrc(A.cout + so, SB);
    sfor<0, HD>::run([&](auto jc) {
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
        if constexpr (MODE == PW_NORM) {
          nacc += norm2(bload_nt<R>(rX, vt, o));
        } else if constexpr (MODE == PW_SCALE) {
          const double s = A.scale[n];
          const cpx<R> x = bload_nt<R>(rX, vt, o);
          A.out64[so + int64_t(g) * SS + c * M + p] = cpx<double>{s * double(x.x), s * double(x.y)};
        } else {  // PW_PRED
          const R s = R(A.scale[n]);
          const cpx<R> phi = s * bload_nt<R>(rX, vt, o);
          cpx<R> pp = phi, cc = phi;
          sfor<0, HD>::run([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const cpx<R> f = bload_nt<R>(rH[j], vt, o);
            if constexpr (j < NP) pp = pp + R(A.b[j]) * f;
            if constexpr (j + 1 < NQ) cc = cc + R(A.a[j + 1]) * f;
          });
          bstore_nt<R>(pp, rX, vt, o);
          bstore_nt<R>(cc, rC, vt, o);
          nacc += norm2(pp);
        }
      }
    }
  }
  if (MODE != PW_SCALE && A.nrm_part) {
    const double t = block_sum<TB>(nacc, red);
    if (tid == 0) A.nrm_part[n * A.nrm_stride + g] = t;
  }
  }
}

// ---------------------------------------------------------------------------
// Kinetic and current densities (measurement path).  For one axis, one
// thread owns one line of one state: D1 with the Nyquist bin zeroed and the
// Nyquist amplitude c give per state and site
//   tau_n += w_v (|D1 v|^2 + (pi/d)^2 |c_v|^2) + w_u (|D1 u|^2 + (pi/d)^2 |c_u|^2)
//   j_n   += w_v Im(v D1 v^*) - w_u Im(u D1 u^*)
// into per-state scratch (tau_s [cs][M], j_s [cs][3][M]); AXIS 0 initialises.
template <typename R, int NL, int AXIS, int TBG>
__global__ __launch_bounds__(TBG) void k_grad_axis(
    const cpx<R>* __restrict__ X, int64_t n0, int64_t nchunk, int64_t M, int64_t stride,
    int64_t inner, const double* __restrict__ scale, const double* __restrict__ wu,
    const double* __restrict__ wv, double kscale, double nyq2, double* __restrict__ tau_s,
    double* __restrict__ j_s) {
  const int64_t nlines = M / NL;
  const int64_t l = int64_t(blockIdx.x) * TBG + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (l >= nlines || c >= nchunk) return;
  const int64_t n = n0 + c;
  // line l -> first site: lines enumerate (outer, inner) with the axis between
  const int64_t outer = l / inner, in = l - outer * inner;
  const int64_t site0 = outer * inner * NL + in;
  const R s = R(scale[n]);
  const double fu = wu[n], fv = wv[n];
  double* ts = tau_s + c * M + site0;
  double* js = j_s + (c * 3 + AXIS) * M + site0;
  constexpr int ES = sizeof(cpx<R>);
  const bi32x4 rX = make_rsrc(X + n * 2 * M, uint32_t(2 * M * ES));
  const int vo = int(site0) * ES;
#pragma unroll 1
  for (int comp = 0; comp < 2; ++comp) {
    const double w = comp ? fv : fu;
    const double sg = comp ? 1.0 : -1.0;
    cpx<R> d[NL], ny;
#pragma unroll
    for (int k = 0; k < NL; ++k) d[k] = s * bload<R>(rX, vo, int(comp * M + k * stride) * ES);
    first_derivative<NL>(d, R(kscale), ny);
    const double cn = nyq2 * norm2(ny);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const double tv = w * (norm2(d[k]) + cn);
      // Im(f (D1 f)^*) = f.y d.x - f.x d.y  (f re-read from cache)
      const cpx<R> f = s * bload<R>(rX, vo, int(comp * M + k * stride) * ES);
      const double jv = sg * w * (double(f.y) * double(d[k].x) - double(f.x) * double(d[k].y));
      if (AXIS == 0 && comp == 0) {
        ts[k * stride] = tv;
      } else {
        ts[k * stride] += tv;
      }
      if (comp == 0) {
        js[k * stride] = jv;
      } else {
        js[k * stride] += jv;
      }
    }
  }
}

// plane-wave states of the uniform H; one block row per state.  both = 0:
// the E > 0 state of every listed momentum (xi = k^2/2 + hshift,
// E = sqrt(xi^2 + Delta^2), u = sqrt((1 + xi/E)/2), v = sqrt((1 - xi/E)/2)).
// both = 1 (spin-imbalanced uniform problem, both branches): for the i-th
// momentum states 2i and 2i+1, (u, v) at dshift + E and (-v, u) at
// dshift - E, with hshift = U - (mu_a + mu_b)/2 and dshift = -(mu_a - mu_b)/2
// (the reduced matrix of the momentum is dshift + the symmetric one).
template <typename R>
__global__ void k_plane_waves(int64_t M, int64_t nstates, int nx, int ny, int nz, const int32_t* __restrict__ kidx,
                              double hshift, double delta0, double kx, double ky, double kz,
                              double invsqrtV, cpx<R>* __restrict__ X, double* __restrict__ E, int both,
                              double dshift) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  for (int64_t n = blockIdx.y; n < nstates; n += gridDim.y) {
  const int64_t i = both ? n / 2 : n;
  const bool minus = both && (n % 2 == 1);
  const int lx = kidx[3 * i], ly = kidx[3 * i + 1], lz = kidx[3 * i + 2];
  const int mx = lx < nx / 2 ? lx : lx - nx, my = ly < ny / 2 ? ly : ly - ny,
            mz = lz < nz / 2 ? lz : lz - nz;
  const double k2 = kx * kx * mx * mx + ky * ky * my * my + kz * kz * mz * mz;
  const double xi = 0.5 * k2 + hshift;
  const double e = sqrt(xi * xi + delta0 * delta0);
  const double uk0 = sqrt(0.5 * (1.0 + xi / e)), vk0 = sqrt(0.5 * (1.0 - xi / e));
  const double uk = minus ? -vk0 : uk0, vk = minus ? uk0 : vk0;
  if (r == 0) E[n] = both ? (minus ? dshift - e : dshift + e) : e;
  if (r >= M) continue;
  const int ix = int(r / (int64_t(ny) * nz)), iy = int((r / nz) % ny), iz = int(r % nz);
  // phase / (2 pi) reduced exactly with integers
  const long fx = ((long(lx) * ix) % nx), fy = ((long(ly) * iy) % ny), fz = ((long(lz) * iz) % nz);
  const double frac = double(fx) / nx + double(fy) / ny + double(fz) / nz;
  double sn, cs;
  sincospi(2.0 * frac, &sn, &cs);
  X[n * 2 * M + r] = cpx<R>{R(uk * cs * invsqrtV), R(uk * sn * invsqrtV)};
  X[n * 2 * M + M + r] = cpx<R>{R(vk * cs * invsqrtV), R(vk * sn * invsqrtV)};
  }
}

// vortex imprint: gauge rotation of both components by theta/2,
// u <- e^{i theta/2} u, v <- e^{-i theta/2} v (nu, hence Delta, gains
// e^{i theta}; the partner map of the spin-symmetric reduction commutes
// with it)
template <typename R>
__global__ void k_imprint(int64_t M, int64_t nstates, const double* __restrict__ theta,
                          cpx<R>* __restrict__ X) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  double sn, cs;
  sincos(0.5 * theta[r], &sn, &cs);
  for (int64_t n = blockIdx.y; n < nstates; n += gridDim.y) {
    const cpx<R> u = X[n * 2 * M + r], v = X[n * 2 * M + M + r];
    const double ur = u.x, ui = u.y, vr = v.x, vi = v.y;
    X[n * 2 * M + r] = cpx<R>{R(ur * cs - ui * sn), R(ur * sn + ui * cs)};
    X[n * 2 * M + M + r] = cpx<R>{R(vr * cs + vi * sn), R(vi * cs - vr * sn)};
  }
}

// D2 of a real field on an N-point periodic axis (N <= 256, one workgroup):
// out = Re 1/N sum_k (-k^2) f~_k exp(2 pi i k z / N), f~ by direct sums,
// the Nyquist mode kept (Eq. D2); f also converted to the context precision.
template <typename R>
__global__ __launch_bounds__(256) void k_field_d2(int N, double dz, const double* __restrict__ f,
                                                  R* __restrict__ fout, R* __restrict__ out) {
  __shared__ double fr[256], fi[256];
  const int t = threadIdx.x;
  if (t < N) {
    double re = 0.0, im = 0.0;
    for (int z = 0; z < N; ++z) {
      double s_, c_;
      sincos(-2.0 * kPi * double((int64_t(t) * z) % N) / N, &s_, &c_);
      re += f[z] * c_;
      im += f[z] * s_;
    }
    fr[t] = re;
    fi[t] = im;
  }
  __syncthreads();
  if (t >= N) return;
  double acc = 0.0;
  for (int k = 0; k < N; ++k) {
    const double km = 2.0 * kPi / (N * dz) * double(k < N / 2 ? k : k - N);
    double s_, c_;
    sincos(2.0 * kPi * double((int64_t(k) * t) % N) / N, &s_, &c_);
    acc += -km * km * (fr[k] * c_ - fi[k] * s_);
  }
  out[t] = R(acc / N);
  fout[t] = R(f[t]);
}

// host FP64 states -> context precision (and back)
template <typename R>
__global__ void k_convert_in(int64_t count, const cpx<double>* __restrict__ in, cpx<R>* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < count) out[i] = cpx<R>{R(in[i].x), R(in[i].y)};
}

}  // namespace tdslda
