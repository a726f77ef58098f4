// Host-side check of the in-register DFT templates: prints, for every
// supported length, the max deviation of the forward DFT from the direct
// O(N^2) sum, and of the second / first derivative from the k-space
// definitions (evaluated here by the direct sum as well).
#include <cmath>
#include <cstdio>
#include <random>
#include "../../paper_2602_08982_amd/csrc/fft.h"

using namespace tdslda;

template <int N>
static double check() {
  std::mt19937_64 g(N);
  std::normal_distribution<double> nd;
  cpx<double> a[N], out[N];
  for (int j = 0; j < N; ++j) a[j] = {nd(g), nd(g)};
  dft_natural<N, -1>(a, out);
  double err = 0, mx = 0;
  for (int k = 0; k < N; ++k) {
    long double re = 0, im = 0;
    for (int j = 0; j < N; ++j) {
      long double t = -2.0L * 3.141592653589793238462643383279503L * (long double)((j * k) % N) / N;
      re += a[j].x * cosl(t) - a[j].y * sinl(t);
      im += a[j].x * sinl(t) + a[j].y * cosl(t);
    }
    err = std::fmax(err, std::hypot(out[k].x - (double)re, out[k].y - (double)im));
    mx = std::fmax(mx, std::hypot((double)re, (double)im));
  }
  err /= mx;
  // second derivative with L = N * 0.7
  double L = N * 0.7, ks = 2 * M_PI / L;
  cpx<double> b[N];
  for (int j = 0; j < N; ++j) b[j] = a[j];
  double ksd = second_derivative<N>(b, ks * ks);
  double err2 = 0, mx2 = 0;
  for (int x = 0; x < N; ++x) {
    double re = 0, im = 0;
    for (int k = 0; k < N; ++k) {
      int m = k < N / 2 ? k : k - N;
      double f = -(ks * m) * (ks * m) / N;
      double t = 2 * M_PI * double(k) * x / N;
      re += f * (out[k].x * std::cos(t) - out[k].y * std::sin(t));
      im += f * (out[k].x * std::sin(t) + out[k].y * std::cos(t));
    }
    err2 = std::fmax(err2, std::hypot(b[x].x - re, b[x].y - im));
    mx2 = std::fmax(mx2, std::hypot(re, im));
  }
  err2 /= mx2;
  cpx<double> c[N], ny;
  for (int j = 0; j < N; ++j) c[j] = a[j];
  first_derivative<N>(c, ks, ny);
  double err1 = std::hypot(ny.x - out[N / 2].x / N, ny.y - out[N / 2].y / N), mx1 = 0;
  for (int x = 0; x < N; ++x) {
    double re = 0, im = 0;
    for (int k = 0; k < N; ++k) {
      if (k == N / 2) continue;
      int m = k < N / 2 ? k : k - N;
      double t = 2 * M_PI * double(k) * x / N;
      // i*k*X_k/N
      double xr = -ks * m * out[k].y / N, xi = ks * m * out[k].x / N;
      re += xr * std::cos(t) - xi * std::sin(t);
      im += xr * std::sin(t) + xi * std::cos(t);
    }
    err1 = std::fmax(err1, std::hypot(c[x].x - re, c[x].y - im));
    mx1 = std::fmax(mx1, std::hypot(re, im));
  }
  err1 = mx1 > 0 ? err1 / mx1 : err1;
  cpx<double> e[N];
  for (int j = 0; j < N; ++j) e[j] = a[j];
  double ks2 = kinetic_sum<N>(e), ref = 0;
  for (int k = 0; k < N; ++k) {
    int m = k < N / 2 ? k : k - N;
    ref += double(m) * m * (out[k].x * out[k].x + out[k].y * out[k].y);
  }
  double errk = std::fmax(std::fabs(ks2 - ref) / ref, std::fabs(ksd - ref) / ref);
  std::printf("N=%d dft=%.3e d2=%.3e d1=%.3e kin=%.3e\n", N, err, err2, err1, errk);
  return std::fmax(std::fmax(err, err2), std::fmax(err1, errk));
}

// lane-pair form: two lanes simulated by two arrays, the exchange by
// swapping them; forward against the direct sum (the even lane holding
// frequency f, the odd one f + N/2 at position p), wave numbers, and the
// inverse back to the samples
template <int N>
static double check_pair() {
  constexpr int H = N / 2;
  std::mt19937_64 g(N + 1000);
  std::normal_distribution<double> nd;
  cpx<double> a[N], out[N];
  for (int j = 0; j < N; ++j) a[j] = {nd(g), nd(g)};
  dft_natural<N, -1>(a, out);
  cpx<double> h[2][H], o[2][H];
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < H; ++j) h[b][j] = a[2 * j + b];
  for (int b = 0; b < 2; ++b) {
    fwd<H>(h[b]);
    pair_twiddle<N, -1>(h[b], b == 1);
  }
  for (int b = 0; b < 2; ++b)
    for (int p = 0; p < H; ++p) o[b][p] = h[1 - b][p];
  for (int b = 0; b < 2; ++b)
    for (int p = 0; p < H; ++p) h[b][p] = pair_butterfly<H>(h[b][p], o[b][p], b == 1);
  double err = 0, mx = 0;
  int bad_m = 0;
  sfor<0, H>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    for (int b = 0; b < 2; ++b) {
      const int k = freq_of_pos<H>(p) + b * H;
      err = std::fmax(err, std::hypot(h[b][p].x - out[k].x, h[b][p].y - out[k].y));
      mx = std::fmax(mx, std::hypot(out[k].x, out[k].y));
      const int m = pair_wavenum<N, p>(b == 1);
      if (m != wavenum<N>(k) && !(k == H && m == -H)) ++bad_m;
    }
  });
  for (int b = 0; b < 2; ++b)
    for (int p = 0; p < H; ++p) o[b][p] = h[1 - b][p];
  for (int b = 0; b < 2; ++b) {
    for (int p = 0; p < H; ++p) h[b][p] = pair_butterfly<H>(h[b][p], o[b][p], b == 1);
    pair_twiddle<N, +1>(h[b], b == 1);
    inv<H>(h[b]);
  }
  double erri = 0;
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < H; ++j)
      erri = std::fmax(erri, std::hypot(h[b][j].x / N - a[2 * j + b].x, h[b][j].y / N - a[2 * j + b].y));
  std::printf("pair N=%d dft=%.3e inverse=%.3e wavenumbers %s\n", N, err / mx, erri, bad_m ? "WRONG" : "ok");
  return bad_m ? 1.0 : std::fmax(err / mx, erri);
}

int main() {
  double e = 0;
  e = std::fmax(e, check_pair<4>());
  e = std::fmax(e, check_pair<6>());
  e = std::fmax(e, check_pair<8>());
  e = std::fmax(e, check_pair<12>());
  e = std::fmax(e, check_pair<16>());
  e = std::fmax(e, check_pair<24>());
  e = std::fmax(e, check_pair<32>());
  e = std::fmax(e, check_pair<48>());
  e = std::fmax(e, check<2>());
  e = std::fmax(e, check<4>());
  e = std::fmax(e, check<6>());
  e = std::fmax(e, check<8>());
  e = std::fmax(e, check<12>());
  e = std::fmax(e, check<16>());
  e = std::fmax(e, check<24>());
  e = std::fmax(e, check<32>());
  e = std::fmax(e, check<48>());
  e = std::fmax(e, check<64>());
  e = std::fmax(e, check<96>());
  e = std::fmax(e, check<128>());
  e = std::fmax(e, check<256>());
  std::printf("max %.3e\n", e);
  return e < 1e-13 ? 0 : 1;
}
