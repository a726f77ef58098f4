// In-register complex DFT of compile-time length N = 2^a 3^b, used for the
// spectral derivatives of the lattice (one thread owns one line of a
// state).  All indices and twiddles are compile-time constants, so the data
// stays in VGPRs and the twiddles fold into literal operands.
//
// Also compiles for the host (used by a CPU unit test of the transforms).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace tdslda {

template <typename R>
struct cpx {
  R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.x, -a.y}; }
// multiply by +i
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_i(cpx<R> a) { return {-a.y, a.x}; }

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2*pi*p/q (argument reduced to [0, pi/4] with
// integer arithmetic, then a Taylor series evaluated in double precision)
namespace ct {
constexpr double kHalfPi = 1.57079632679489661923132169163975;

constexpr double sin_series(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// returns {cos, sin} of 2*pi*p/q
struct cs {
  double c, s;
};
constexpr cs cossin(long p, long q) {
  long r = ((p % q) + q) % q;      // angle 2*pi*r/q in [0, 2*pi)
  long a = 4 * r;                  // = quadrant units * q
  long quad = a / q;               // 0..3
  long rem = a - quad * q;         // angle within quadrant = (pi/2) rem/q
  bool swap = 2 * rem > q;         // reflect about pi/4
  long m = swap ? q - rem : rem;
  double phi = kHalfPi * double(m) / double(q);
  double s0 = sin_series(phi), c0 = cos_series(phi);
  double sp = swap ? c0 : s0, cp = swap ? s0 : c0;  // sin, cos of the in-quadrant angle
  switch (quad) {
    case 0: return {cp, sp};
    case 1: return {-sp, cp};
    case 2: return {-cp, -sp};
    default: return {sp, -cp};
  }
}
}  // namespace ct

// x * exp(SIGN * 2*pi*i * P / N)
template <int P, int N, int SIGN, typename R>
__host__ __device__ __forceinline__ cpx<R> twiddle(cpx<R> x) {
  constexpr int p = ((P % N) + N) % N;
  if constexpr (p == 0) {
    return x;
  } else if constexpr (4 * p == N) {  // quarter turn
    return SIGN > 0 ? mul_i(x) : cpx<R>{x.y, -x.x};
  } else if constexpr (2 * p == N) {
    return {-x.x, -x.y};
  } else if constexpr (4 * p == 3 * N) {
    return SIGN > 0 ? cpx<R>{x.y, -x.x} : mul_i(x);
  } else {
    constexpr ct::cs w = ct::cossin(p, N);
    constexpr R c = R(w.c);
    constexpr R s = R(SIGN * w.s);
    return {x.x * c - x.y * s, x.x * s + x.y * c};
  }
}

template <int I, int E>
struct sfor {
  template <class F>
  __host__ __device__ __forceinline__ static void run(F&& f) {
    f(std::integral_constant<int, I>{});
    sfor<I + 1, E>::run(f);
  }
};
template <int E>
struct sfor<E, E> {
  template <class F>
  __host__ __device__ __forceinline__ static void run(F&&) {}
};

template <int N>
constexpr int radix_of() {
  return (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : (N % 3 == 0) ? 3 : 0;
}

// r-point DFT of t[] in place (sign SIGN), r in {2, 3, 4}
template <int r, int SIGN, typename R>
__host__ __device__ __forceinline__ void small_dft(cpx<R> (&t)[r]) {
  if constexpr (r == 2) {
    cpx<R> a = t[0] + t[1], b = t[0] - t[1];
    t[0] = a;
    t[1] = b;
  } else if constexpr (r == 4) {
    cpx<R> a = t[0] + t[2], b = t[0] - t[2];
    cpx<R> c = t[1] + t[3], d = t[1] - t[3];
    cpx<R> wd = SIGN > 0 ? mul_i(d) : cpx<R>{d.y, -d.x};  // (SIGN i) * d
    t[0] = a + c;
    t[1] = b + wd;
    t[2] = a - c;
    t[3] = b - wd;
  } else {
    static_assert(r == 3, "radix");
    constexpr R h = R(0.86602540378443864676372317075294);  // sqrt(3)/2
    cpx<R> a = t[1] + t[2], b = t[1] - t[2];
    cpx<R> base = t[0] - R(0.5) * a;
    cpx<R> rb = R(SIGN) * h * mul_i(b);
    t[0] = t[0] + a;
    t[1] = base + rb;
    t[2] = base - rb;
  }
}

// In-place decimation-in-frequency DFT (sign SIGN) of a[N]: natural order in,
// digit-reversed order out (position p holds frequency freq_of_pos<N>(p)).
// Stage on blocks of length L with radix r: for every block and j < L/r the
// r inputs a[j + q L/r] go through an r-point DFT and the k-th output is
// multiplied by w_L^(SIGN j k) and stored at a[j + k L/r].
template <int N, int L, int SIGN, typename R>
__host__ __device__ __forceinline__ void dif_stages(cpx<R> (&a)[N]) {
  if constexpr (L > 1) {
    constexpr int r = radix_of<L>();
    static_assert(r != 0, "line length must be 2^a 3^b");
    constexpr int Q = L / r;
    sfor<0, N / L>::run([&](auto bc) {
      constexpr int b0 = decltype(bc)::value * L;
      sfor<0, Q>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        cpx<R> t[r];
        sfor<0, r>::run([&](auto qc) { t[decltype(qc)::value] = a[b0 + j + decltype(qc)::value * Q]; });
        small_dft<r, SIGN>(t);
        sfor<0, r>::run([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          a[b0 + j + k * Q] = twiddle<j * k, L, SIGN>(t[k]);
        });
      });
    });
    dif_stages<N, Q, SIGN>(a);
  }
}

// In-place decimation-in-time DFT (sign SIGN): digit-reversed order in (as
// produced by dif_stages), natural order out.  It is the transposed flow
// graph of dif_stages: stages in reverse order, twiddles before the
// butterflies.
template <int N, int L, int SIGN, typename R>
__host__ __device__ __forceinline__ void dit_stages(cpx<R> (&a)[N]) {
  if constexpr (L > 1) {
    constexpr int r = radix_of<L>();
    constexpr int Q = L / r;
    dit_stages<N, Q, SIGN>(a);
    sfor<0, N / L>::run([&](auto bc) {
      constexpr int b0 = decltype(bc)::value * L;
      sfor<0, Q>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        cpx<R> t[r];
        sfor<0, r>::run([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          t[k] = twiddle<j * k, L, SIGN>(a[b0 + j + k * Q]);
        });
        small_dft<r, SIGN>(t);
        sfor<0, r>::run([&](auto qc) { a[b0 + j + decltype(qc)::value * Q] = t[decltype(qc)::value]; });
      });
    });
  }
}

// frequency held at position p after dif_stages<N>
template <int N>
__host__ __device__ constexpr int freq_of_pos(int p) {
  int L = N, f = 0, mult = 1;
  while (L > 1) {
    int r = (L % 4 == 0) ? 4 : (L % 2 == 0) ? 2 : 3;
    int Q = L / r;
    int k = p / Q;
    p -= k * Q;
    f += mult * k;
    mult *= r;
    L = Q;
  }
  return f;
}

// signed integer wave number of DFT bin j on an N-point periodic axis
template <int N>
__host__ __device__ constexpr int wavenum(int j) {
  return j < N / 2 ? j : j - N;
}
// signed wave number held at position p after dif_stages<N>
template <int N>
__host__ __device__ constexpr int wavenum_at(int p) {
  return wavenum<N>(freq_of_pos<N>(p));
}

// forward / inverse (unnormalised) in place; between them the data are
// digit-reversed
template <int N, typename R>
__host__ __device__ __forceinline__ void fwd(cpx<R> (&a)[N]) { dif_stages<N, N, -1>(a); }
template <int N, typename R>
__host__ __device__ __forceinline__ void inv(cpx<R> (&a)[N]) { dit_stages<N, N, +1>(a); }

// natural-order DFT: out[k] = sum_j a[j] exp(SIGN 2 pi i j k / N)
template <int N, int SIGN, typename R>
__host__ __device__ __forceinline__ void dft_natural(const cpx<R> (&a)[N], cpx<R> (&out)[N]) {
  cpx<R> t[N];
  for (int j = 0; j < N; ++j) t[j] = a[j];
  dif_stages<N, N, SIGN>(t);
  sfor<0, N>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    out[freq_of_pos<N>(p)] = t[p];
  });
}

// Second derivative along a line, in place: IDFT(-k^2 DFT(a)) with the full
// k^2 of every bin including the Nyquist one.  kscale2 = (2*pi/L)^2.
// Returns sum_k m_k^2 |a_k|^2 (integer wave numbers m, unnormalised DFT),
// so that sum_x |d a/dx|^2 = kscale2 * returned / N (Parseval).
template <int N, typename R>
__host__ __device__ __forceinline__ double second_derivative(cpx<R> (&a)[N], R kscale2) {
  fwd<N>(a);
  const R f = -kscale2 / R(N);
  double ks = 0.0;
  sfor<0, N>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int m = wavenum_at<N>(p);
    if constexpr (m != 0) ks += double(m * m) * (double(a[p].x) * double(a[p].x) + double(a[p].y) * double(a[p].y));
    a[p] = (f * R(m * m)) * a[p];
  });
  inv<N>(a);
  return ks;
}

// Forward transform (destroys a) and sum_k m_k^2 |a_k|^2.
template <int N, typename R>
__host__ __device__ __forceinline__ double kinetic_sum(cpx<R> (&a)[N]) {
  fwd<N>(a);
  double acc = 0.0;
  sfor<0, N>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int m = wavenum_at<N>(p);
    if constexpr (m != 0) acc += double(m * m) * (double(a[p].x) * double(a[p].x) + double(a[p].y) * double(a[p].y));
  });
  return acc;
}

// First derivative in place with the Nyquist bin zeroed (the paper's
// odd-derivative rule); nyq = DFT(a)[N/2] / N.  kscale = 2*pi/L.
template <int N, typename R>
__host__ __device__ __forceinline__ void first_derivative(cpx<R> (&a)[N], R kscale, cpx<R>& nyq) {
  fwd<N>(a);
  const R f = kscale / R(N);
  sfor<0, N>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int fq = freq_of_pos<N>(p);
    constexpr int m = wavenum<N>(fq);
    if constexpr (fq == N / 2) {
      nyq = (R(1) / R(N)) * a[p];
      a[p] = cpx<R>{R(0), R(0)};
    } else {
      a[p] = (f * R(m)) * mul_i(a[p]);
    }
  });
  inv<N>(a);
}

// ---------------------------------------------------------------------------
// Lane-pair DFT of even length N: two adjacent lanes (parity b) share one
// line, lane b holding the samples a[2j + b], j < N/2, so that a line needs
// half the registers.  Radix-2 decimation in time across the pair: each lane
// transforms its half (fwd<N/2>: position p holds frequency f =
// freq_of_pos<N/2>(p)), the odd lane multiplies by w_N^-f, the lanes swap
// values and combine, X[f] = E + w^-f O in the even lane and X[f + N/2] =
// E - w^-f O in the odd one.  The inverse runs the flow graph backwards
// (combine, odd-lane twiddle w_N^+f, inv<N/2>), back to the lane's samples.
// The exchange is the only cross-lane step (device: a DPP swap of each
// lane pair); the steps around it also compile for the host.
template <int N, int SIGN, typename R>
__host__ __device__ __forceinline__ void pair_twiddle(cpx<R> (&h)[N / 2], bool odd) {
  constexpr int H = N / 2;
  sfor<0, H>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    const cpx<R> t = twiddle<freq_of_pos<H>(p), N, SIGN>(h[p]);
    // select per scalar (a select of the two values as a whole would take
    // their addresses and keep the array out of registers)
    h[p] = cpx<R>{odd ? t.x : h[p].x, odd ? t.y : h[p].y};
  });
}
// h <- o + h (even lane), o - h (odd lane); o = the partner's h
template <int H, typename R>
__host__ __device__ __forceinline__ cpx<R> pair_butterfly(cpx<R> h, cpx<R> o, bool odd) {
  const R sg = odd ? R(-1) : R(1);
  return cpx<R>{o.x + sg * h.x, o.y + sg * h.y};
}
// signed wave number held at position p by lane parity odd after fwd_pair<N>
template <int N, int P>
__host__ __device__ __forceinline__ int pair_wavenum(bool odd) {
  constexpr int H = N / 2, f = freq_of_pos<H>(P);
  return odd ? f - H : f;
}

// the same at run time for row position q = 2p + b of a line stored by
// lane pairs
template <int N>
__host__ __device__ __forceinline__ int pair_wavenum_at(int q) {
  const int f = freq_of_pos<N / 2>(q >> 1);
  return (q & 1) ? f - N / 2 : f;
}

#ifdef __HIP__
__device__ __forceinline__ float lane_pair_swap(float x) {
  // quad_perm [1, 0, 3, 2]: lanes 2i and 2i + 1 exchange
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_pair_swap(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp(int(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(v >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}
template <typename R>
__device__ __forceinline__ cpx<R> lane_pair_swap(cpx<R> c) {
  return cpx<R>{lane_pair_swap(c.x), lane_pair_swap(c.y)};
}
// both lanes of every pair must be active
template <int N, typename R>
__device__ __forceinline__ void fwd_pair(cpx<R> (&h)[N / 2], bool odd) {
  constexpr int H = N / 2;
  fwd<H>(h);
  pair_twiddle<N, -1>(h, odd);
  sfor<0, H>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    h[p] = pair_butterfly<H>(h[p], lane_pair_swap(h[p]), odd);
  });
}
template <int N, typename R>
__device__ __forceinline__ void inv_pair(cpx<R> (&h)[N / 2], bool odd) {
  constexpr int H = N / 2;
  sfor<0, H>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    h[p] = pair_butterfly<H>(h[p], lane_pair_swap(h[p]), odd);
  });
  pair_twiddle<N, +1>(h, odd);
  inv<H>(h);
}
// second_derivative / first_derivative in the lane-pair form (each lane's
// half of the line in place); nyq = DFT(a)[N/2] / N in both lanes
template <int N, typename R>
__device__ __forceinline__ void second_derivative_pair(cpx<R> (&h)[N / 2], R kscale2, bool odd) {
  fwd_pair<N>(h, odd);
  const R f = -kscale2 / R(N);
  sfor<0, N / 2>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    const R m = R(pair_wavenum<N, p>(odd));
    h[p] = (f * m * m) * h[p];
  });
  inv_pair<N>(h, odd);
}
template <int N, typename R>
__device__ __forceinline__ void first_derivative_pair(cpx<R> (&h)[N / 2], R kscale, bool odd, cpx<R>& nyq) {
  fwd_pair<N>(h, odd);
  // the Nyquist bin is position 0 of the odd lane
  const cpx<R> other = lane_pair_swap(h[0]);
  nyq = (R(1) / R(N)) * cpx<R>{odd ? h[0].x : other.x, odd ? h[0].y : other.y};
  const R f = kscale / R(N);
  sfor<0, N / 2>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    const int m = pair_wavenum<N, p>(odd);
    const R km = (m == -N / 2) ? R(0) : f * R(m);
    h[p] = km * mul_i(h[p]);
  });
  inv_pair<N>(h, odd);
}
#endif

}  // namespace tdslda
