// Checks of the FFT building blocks and the real-to-complex pair-stage bodies,
// built for the host against tests/cpu_fft/hip/hip_runtime.h and run with one
// thread.  References are written out from the definitions (naive DFTs).
// Prints one line per check and exits non-zero on a failure.
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "../../paper_2101_03155_amd/csrc/pair_phases.h"

using namespace ace;
using cd = std::complex<double>;
static int failures = 0;

static void report(const char* what, int n, double err, double tol) {
  const bool ok = err <= tol;
  if (!ok) ++failures;
  std::printf("%-34s N=%3d rel err %.2e (tol %.0e) %s\n", what, n, err, tol, ok ? "ok" : "FAIL");
}

static unsigned lcg(unsigned& s) { return s = s * 1664525u + 1013904223u; }
static double uni(unsigned& s) { return (lcg(s) >> 8) / double(1 << 24) - 0.5; }

template <typename T, int N>
std::vector<cplx<T>> twiddles() {
  std::vector<cplx<T>> tw(N);
  for (int m = 0; m < N; ++m) {
    tw[m].x = T(std::cos(-2.0 * M_PI * m / N));
    tw[m].y = T(std::sin(-2.0 * M_PI * m / N));
  }
  return tw;
}

// One line, both signs, both plan orders, against the naive DFT.
template <typename T, int N, int S, int V>
double line_err() {
  std::vector<cplx<T>> buf(N), tw = twiddles<T, N>();
  std::vector<cd> x(N);
  unsigned s = 12345u + N;
  for (int i = 0; i < N; ++i) {
    x[i] = cd(uni(s), uni(s));
    buf[i].x = T(x[i].real());
    buf[i].y = T(x[i].imag());
  }
  fft_lines<T, N, 1, N, 1, 1, S, false, V>(buf.data(), tw.data(), 0);
  double err = 0, mx = 0;
  for (int k = 0; k < N; ++k) {
    cd acc = 0;
    for (int n = 0; n < N; ++n) acc += x[n] * std::polar(1.0, S * 2.0 * M_PI * double((long(n) * k) % N) / N);
    err = std::max(err, std::abs(acc - cd(buf[k].x, buf[k].y)));
    mx = std::max(mx, std::abs(acc));
  }
  return err / mx;
}

// Inverse body (staged in LDS, or reading the plane from memory) in plan
// order V: N^2 rho in the packed rows of the inverse layout.
template <typename T, int N, int V>
double inverse_err(const std::vector<T>& pi, const std::vector<T>& pj, const std::vector<cplx<T>>& out,
                   const std::vector<cplx<T>>& tw, bool global) {
  constexpr int H = N / 2;
  using Lay = InvLayout<T, N, V>;
  std::vector<cplx<T>> buf(N * (N / 2 + 1));
  for (auto& c : buf) { c.x = T(1e30); c.y = T(-1e30); }
  if (global) body_inv_xy_g<T, N, 1, V>(out.data(), buf.data(), tw.data(), 0);
  else body_inv_xy_r<T, N, 1, V>(out.data(), buf.data(), tw.data(), 0);
  double e2 = 0, m2 = 0;
  for (int l = 0; l < H; ++l)
    for (int x = 0; x < N; ++x) {
      const double r0 = double(pi[l * N + x]) * pj[l * N + x] * N * N;
      const double r1 = double(pi[(l + H) * N + x]) * pj[(l + H) * N + x] * N * N;
      const auto v = buf[Lay::xq(l, x)];
      e2 = std::max(e2, std::max(std::abs(v.x - r0), std::abs(v.y - r1)));
      m2 = std::max(m2, std::max(std::abs(r0), std::abs(r1)));
    }
  return e2 / m2;
}

// Forward in-plane body against the 2D DFT of phi_i phi_j; the inverse body
// must return N^2 rho in the packed rows.
template <typename T, int N>
void check_plane(double tol) {
  constexpr int XS = N / 2 + 1;
  std::vector<T> pi(N * N), pj(N * N);
  unsigned s = 777u + N;
  for (int e = 0; e < N * N; ++e) { pi[e] = T(uni(s)); pj[e] = T(uni(s)); }
  std::vector<cplx<T>> tw = twiddles<T, N>(), buf(N * XS), out(N * XS);
  body_fwd_xy_r<T, N, 1>(pi.data(), pj.data(), out.data(), buf.data(), tw.data(), 0);
  double err = 0, mx = 0;
  for (int ky = 0; ky < N; ++ky)
    for (int kx = 0; kx < XS; ++kx) {
      cd acc = 0;
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x)
          acc += double(pi[y * N + x]) * double(pj[y * N + x]) *
                 std::polar(1.0, -2.0 * M_PI * double((kx * x + ky * y) % N) / N);
      err = std::max(err, std::abs(acc - cd(out[ky * XS + kx].x, out[ky * XS + kx].y)));
      mx = std::max(mx, std::abs(acc));
    }
  report(sizeof(T) == 8 ? "forward in-plane, fp64" : "forward in-plane, fp32", N, err / mx, tol);
  double e2 = 0;
  for (bool g : {false, true})
    e2 = std::max(e2, std::max(inverse_err<T, N, 0>(pi, pj, out, tw, g), inverse_err<T, N, 1>(pi, pj, out, tw, g)));
  report(sizeof(T) == 8 ? "inverse in-plane round trip, fp64" : "inverse in-plane round trip, fp32", N, e2, tol);
}

// z pass (forward z DFT, times v(G), inverse z DFT) over all tiles of a
// slot, ragged last tile included, against the naive transforms; and the
// table-driven pass bitwise equal to the per-element one.
template <typename T, int N>
void check_z(double tol) {
  constexpr int XS = N / 2 + 1, PL = N * XS, TX = own_tx<T, N>();
  constexpr int NT = (PL + TX - 1) / TX;
  std::vector<cplx<T>> spec(N * PL), ref(N * PL), spec2;
  unsigned s = 31u + N;
  for (auto& c : spec) { c.x = T(uni(s)); c.y = T(uni(s)); }
  spec2 = spec;
  KernelParams kp{1, 0.37, 1.0 / (double(N) * N * N), {0.41, 0.43, 0.47}};
  for (int f = 0; f < PL; ++f) {
    std::vector<cd> col(N), hat(N);
    for (int z = 0; z < N; ++z) col[z] = cd(spec[z * PL + f].x, spec[z * PL + f].y);
    for (int k = 0; k < N; ++k) {
      cd acc = 0;
      for (int z = 0; z < N; ++z) acc += col[z] * std::polar(1.0, -2.0 * M_PI * double((k * z) % N) / N);
      hat[k] = acc * double(kernel_value<T, N>(kp, f % XS, f / XS, k));
    }
    for (int z = 0; z < N; ++z) {
      cd acc = 0;
      for (int k = 0; k < N; ++k) acc += hat[k] * std::polar(1.0, 2.0 * M_PI * double((k * z) % N) / N);
      ref[z * PL + f] = cplx<T>{T(acc.real()), T(acc.imag())};
    }
  }
  // the library's table: folded y and z frequencies, [zq][yq][kx]
  constexpr int H = N / 2 + 1;
  std::vector<T> vt(H * H * XS);
  for (int e = 0; e < H * H * XS; ++e) vt[e] = kernel_value<T, N>(kp, e % XS, (e / XS) % H, e / (XS * H));
  std::vector<cplx<T>> buf(N * TX), tw = twiddles<T, N>();
  double es = 0, red[4];
  for (int t = 0; t < NT; ++t) {
    body_conv_z_r<T, N, TX, 1>(spec.data(), t * TX, kp, buf.data(), tw.data(), 0, true, &es, red, nullptr);
    body_conv_z_r<T, N, TX, 1>(spec2.data(), t * TX, kp, buf.data(), tw.data(), 0, true, &es, red, vt.data());
  }
  double err = 0, mx = 0;
  bool same = true;
  for (int e = 0; e < N * PL; ++e) {
    err = std::max(err, std::abs(cd(spec[e].x, spec[e].y) - cd(ref[e].x, ref[e].y)));
    mx = std::max(mx, std::abs(cd(ref[e].x, ref[e].y)));
    same = same && spec[e].x == spec2[e].x && spec[e].y == spec2[e].y;
  }
  report(sizeof(T) == 8 ? "z pass with v(G), fp64" : "z pass with v(G), fp32", N, err / mx, tol);
  report("z pass: table == per-element v(G)", N, same ? 0.0 : 1.0, 0.0);
}

template <int N>
void lines() {
  const double e = std::max(std::max(line_err<double, N, -1, 0>(), line_err<double, N, 1, 0>()),
                            std::max(line_err<double, N, -1, 1>(), line_err<double, N, 1, 1>()));
  report("FFT lines, fp64, both signs/orders", N, e, 4e-15);
  report("FFT lines, fp32", N, std::max(line_err<float, N, -1, 0>(), line_err<float, N, 1, 1>()), 5e-7);
}

int main() {
  lines<8>(); lines<12>(); lines<16>(); lines<20>(); lines<24>(); lines<32>(); lines<48>(); lines<64>();
  lines<80>(); lines<96>(); lines<100>(); lines<108>(); lines<120>(); lines<160>();
  check_plane<double, 12>(1e-13); check_plane<double, 16>(1e-13); check_plane<double, 24>(1e-13);
  check_plane<double, 32>(1e-13); check_plane<double, 64>(1e-13); check_plane<double, 96>(1e-13);
  check_plane<float, 20>(1e-5); check_plane<float, 96>(1e-5);
  check_z<double, 12>(1e-13); check_z<double, 16>(1e-13); check_z<double, 20>(1e-13);
  check_z<float, 24>(1e-5); check_z<float, 20>(1e-5);
  return failures ? 1 : 0;
}
