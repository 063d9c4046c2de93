// Learned pair screener: features, MLP training and inference, budgeted
// selection.
//
// The screening criterion of Sec. Theory keeps a pair when the overlap
// integral of |phi_i phi_j| exceeds a fixed threshold.  The learned form
// instead predicts each pair's exchange contribution |e_ij| from five
// features and drops the pairs with the smallest predictions while their
// predicted sum stays within an E_x error budget.
//
// Features of pair (i, j): minimum-image distance of the periodic centroids of
// |phi|^2, the smaller and the larger spread, log10 of dV sum |phi_i||phi_j|
// and log10 of dV sum phi_i^2 phi_j^2.
//
// Model (FP32): 5 -> 64 -> 64 -> 1 with tanh, inputs and target standardized
// by statistics stored with the weights.  Flat layout: W1[64][5], b1[64],
// W2[64][64], b2[64], w3[64], b3, then xmean[5], xstd[5], tmean, tstd,
// xmin[5], xmax[5].  Training minimizes the mean squared error of the
// standardized log10 |e_ij| with Adam; per-minibatch gradients are sums over
// samples in a fixed order (no atomics), so training is deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ace_internal.h"

namespace ace {

constexpr int NIN = 5, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPAR = OB3 + 1;
constexpr int OXM = NPAR, OXS = OXM + NIN, OTM = OXS + NIN, OTS = OTM + 1, OXMIN = OTS + 1, OXMAX = OXMIN + NIN,
              NMODEL = OXMAX + NIN;
static_assert(NPAR == 4609, "parameter count");
static_assert(NMODEL == 4631, "model size");

// ---------------------------------------------------------------- orbital moments
// Per (orbital, z-plane): the plane's total |phi|^2 and its row (y) and column
// (x) sums; pz[orb][z], py[orb][z][y], px[orb][z][x].
__global__ __launch_bounds__(256) void k_plane_marginals(const double* __restrict__ phi, int n, double* __restrict__ pz,
                                                         double* __restrict__ py, double* __restrict__ px) {
  // one read of the plane: wave w takes rows y = w, w + 4, ...; lanes read the
  // row coalesced, its sum comes from a shuffle reduction, and each lane keeps
  // its columns' partial sums, combined over the waves in LDS at the end
  constexpr int CPL = 4;  // columns per lane (n <= 256)
  const int z = blockIdx.x, orb = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t ng = int64_t(n) * n * n;
  const double* P = phi + int64_t(orb) * ng + int64_t(z) * n * n;
  __shared__ double col[4][256];
  double cs[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) cs[c] = 0.0;
  for (int y = wv; y < n; y += 4) {
    double rs = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int x = lane + 64 * c;
      if (x < n) {
        const double v = P[y * n + x];
        cs[c] += v * v;
        rs += v * v;
      }
    }
    for (int off = 32; off > 0; off >>= 1) rs += __shfl_down(rs, off, 64);
    if (lane == 0) py[(int64_t(orb) * n + z) * n + y] = rs;
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) col[wv][lane + 64 * c] = cs[c];
  __syncthreads();
  double tot = 0.0;
  for (int x = tid; x < n; x += 256) {
    const double s = col[0][x] + col[1][x] + col[2][x] + col[3][x];
    px[(int64_t(orb) * n + z) * n + x] = s;
    tot += s;
  }
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_down(tot, off, 64);
  __syncthreads();
  if (lane == 0) col[0][wv] = tot;
  __syncthreads();
  if (tid == 0) pz[int64_t(orb) * n + z] = col[0][0] + col[0][1] + col[0][2] + col[0][3];
}

// out[orb][zs][ys][xs] = phi[orb][s zs][s ys][s xs]: the grid subsampled by
// the stride s per axis (m = n / s points per axis).
__global__ void k_subsample(const double* __restrict__ phi, int norb, int n, int st, double* __restrict__ out) {
  const int m = n / st;
  const int64_t tot = int64_t(norb) * m * m * m;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int xs = int(e % m);
    int64_t r = e / m;
    const int ys = int(r % m);
    r /= m;
    const int zs = int(r % m);
    const int64_t orb = r / m;
    out[e] = phi[((orb * n + int64_t(zs) * st) * n + int64_t(ys) * st) * n + int64_t(xs) * st];
  }
}

// Per orbital: marginals along each axis, periodic centroid (argument of the
// first Fourier coefficient of the marginal) and spread with minimum-image
// displacements.  cen[orb][3] (x, y, z), spr[orb].
__global__ __launch_bounds__(256) void k_centroids(const double* __restrict__ pz, const double* __restrict__ py,
                                                   const double* __restrict__ px, int n, double L, double dV,
                                                   double* __restrict__ cen, double* __restrict__ spr) {
  const int orb = blockIdx.x, tid = threadIdx.x;
  __shared__ double m[3][512];
  __shared__ double c3[3];
  for (int a = tid; a < n; a += 256) {
    double sx = 0.0, sy = 0.0;
    for (int z = 0; z < n; ++z) {
      sx += px[(int64_t(orb) * n + z) * n + a];
      sy += py[(int64_t(orb) * n + z) * n + a];
    }
    m[0][a] = sx;
    m[1][a] = sy;
    m[2][a] = pz[int64_t(orb) * n + a];
  }
  __syncthreads();
  const double two_pi = 6.283185307179586476925286766559005768;
  if (tid < 3) {
    double cs = 0.0, sn = 0.0;
    for (int a = 0; a < n; ++a) {
      const double ang = two_pi * double(a) / double(n);
      cs += m[tid][a] * cos(ang);
      sn += m[tid][a] * sin(ang);
    }
    double c = atan2(sn, cs) * L / two_pi;
    c = c - L * floor(c / L);
    c3[tid] = c;
    cen[orb * 3 + tid] = c;
  }
  __syncthreads();
  if (tid == 0) {
    double s2 = 0.0;
    for (int ax = 0; ax < 3; ++ax)
      for (int a = 0; a < n; ++a) {
        double d = double(a) * L / double(n) - c3[ax];
        d -= L * rint(d / L);
        s2 += m[ax][a] * d * d;
      }
    spr[orb] = sqrt(s2 * dV);
  }
}

// Pair t -> (i, j), i <= j, row-major over the upper triangle.
__device__ __forceinline__ void tri_ij(int64_t t, int n, int& i, int& j) {
  const double a = 2.0 * n + 1.0;
  i = int((a - sqrt(a * a - 8.0 * double(t))) * 0.5);
  while (i > 0 && int64_t(i) * n - int64_t(i) * (i - 1) / 2 > t) --i;
  while (int64_t(i + 1) * n - int64_t(i + 1) * i / 2 <= t) ++i;
  j = i + int(t - (int64_t(i) * n - int64_t(i) * (i - 1) / 2));
}

// Features of listed pairs (pairs != nullptr) or of every pair i <= j.
__global__ void k_pair_features(const int32_t* __restrict__ pairs, int64_t np, int n, const double* __restrict__ cen,
                                const double* __restrict__ spr, const double* __restrict__ O,
                                const double* __restrict__ P, double L, float* __restrict__ f) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < np; t += int64_t(gridDim.x) * blockDim.x) {
    int i, j;
    if (pairs) { i = pairs[2 * t]; j = pairs[2 * t + 1]; }
    else tri_ij(t, n, i, j);
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double d = cen[i * 3 + a] - cen[j * 3 + a];
      d -= L * rint(d / L);
      d2 += d * d;
    }
    const double o = O[int64_t(i) * n + j], p = P[int64_t(i) * n + j];
    float* out = f + t * NIN;
    out[0] = float(sqrt(d2));
    out[1] = float(fmin(spr[i], spr[j]));
    out[2] = float(fmax(spr[i], spr[j]));
    out[3] = float(log10(fmax(o, 1e-30)));
    out[4] = float(log10(fmax(p, 1e-30)));
  }
}

// ---------------------------------------------------------------- MLP
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Glorot-uniform weights from a counter-based generator, zero biases, unit
// standardization.
__global__ void k_mlp_init(float* __restrict__ m, uint64_t seed) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NMODEL; e += gridDim.x * blockDim.x) {
    const double u = double(splitmix64(seed * 0x100000001B3ull + uint64_t(e)) >> 11) * (1.0 / 9007199254740992.0);
    float v = 0.f;
    if (e < OB1) v = float((2 * u - 1) * sqrt(6.0 / (NIN + NH)));
    else if (e >= OW2 && e < OB2) v = float((2 * u - 1) * sqrt(6.0 / (NH + NH)));
    else if (e >= OW3 && e < OB3) v = float((2 * u - 1) * sqrt(6.0 / (NH + 1)));
    else if (e >= OXS && e < OXS + NIN) v = 1.f;
    else if (e == OTS) v = 1.f;
    m[e] = v;
  }
}

// Per block: sums of x, x^2, min, max per feature and of t, t^2 (FP64).
__global__ __launch_bounds__(256) void k_stats_partial(const float* __restrict__ x, const float* __restrict__ t,
                                                       int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double acc[4 * NIN + 2];
  for (int k = 0; k < NIN; ++k) { acc[k] = 0; acc[NIN + k] = 0; acc[2 * NIN + k] = 1e300; acc[3 * NIN + k] = -1e300; }
  acc[4 * NIN] = acc[4 * NIN + 1] = 0;
  for (int64_t s = blockIdx.x * int64_t(256) + threadIdx.x; s < n; s += int64_t(gridDim.x) * 256) {
    for (int k = 0; k < NIN; ++k) {
      const double v = x[s * NIN + k];
      acc[k] += v; acc[NIN + k] += v * v;
      acc[2 * NIN + k] = fmin(acc[2 * NIN + k], v); acc[3 * NIN + k] = fmax(acc[3 * NIN + k], v);
    }
    acc[4 * NIN] += t[s]; acc[4 * NIN + 1] += double(t[s]) * t[s];
  }
  for (int q = 0; q < 4 * NIN + 2; ++q) {
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) {
        const double a = red[threadIdx.x], b = red[threadIdx.x + h];
        red[threadIdx.x] = (q >= 2 * NIN && q < 3 * NIN) ? fmin(a, b) : (q >= 3 * NIN && q < 4 * NIN) ? fmax(a, b) : a + b;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * (4 * NIN + 2) + q] = red[0];
    __syncthreads();
  }
}

__global__ void k_stats_final(const double* __restrict__ part, int nb, int64_t n, float* __restrict__ m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc[4 * NIN + 2];
  for (int q = 0; q < 4 * NIN + 2; ++q) acc[q] = (q >= 2 * NIN && q < 3 * NIN) ? 1e300 : (q >= 3 * NIN && q < 4 * NIN) ? -1e300 : 0.0;
  for (int b = 0; b < nb; ++b)
    for (int q = 0; q < 4 * NIN + 2; ++q) {
      const double v = part[b * (4 * NIN + 2) + q];
      acc[q] = (q >= 2 * NIN && q < 3 * NIN) ? fmin(acc[q], v) : (q >= 3 * NIN && q < 4 * NIN) ? fmax(acc[q], v) : acc[q] + v;
    }
  for (int k = 0; k < NIN; ++k) {
    const double mu = acc[k] / double(n);
    const double var = acc[NIN + k] / double(n) - mu * mu;
    m[OXM + k] = float(mu);
    m[OXS + k] = float(sqrt(fmax(var, 1e-12)));
    m[OXMIN + k] = float(acc[2 * NIN + k]);
    m[OXMAX + k] = float(acc[3 * NIN + k]);
  }
  const double mu = acc[4 * NIN] / double(n);
  m[OTM] = float(mu);
  m[OTS] = float(sqrt(fmax(acc[4 * NIN + 1] / double(n) - mu * mu, 1e-12)));
}

// Prediction (de-standardized target, log10 |e|) of every sample; with clamp
// the features are first clipped to the training ranges.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ model, const float* __restrict__ x,
                                                     int64_t n, int clamp, float* __restrict__ y) {
  __shared__ float w[NMODEL];
  for (int e = threadIdx.x; e < NMODEL; e += 256) w[e] = model[e];
  __syncthreads();
  for (int64_t s = blockIdx.x * int64_t(256) + threadIdx.x; s < n; s += int64_t(gridDim.x) * 256) {
    float xs[NIN];
    for (int k = 0; k < NIN; ++k) {
      float v = x[s * NIN + k];
      if (clamp) v = fminf(fmaxf(v, w[OXMIN + k]), w[OXMAX + k]);
      xs[k] = (v - w[OXM + k]) / w[OXS + k];
    }
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      float a = w[OB1 + j];
#pragma unroll
      for (int k = 0; k < NIN; ++k) a += w[OW1 + j * NIN + k] * xs[k];
      h1[j] = tanhf(a);
    }
    float out = w[OB3];
    for (int j = 0; j < NH; ++j) {
      float a = w[OB2 + j];
#pragma unroll
      for (int k = 0; k < NH; ++k) a += w[OW2 + j * NH + k] * h1[k];
      out += w[OW3 + j] * tanhf(a);
    }
    y[s] = w[OTM] + w[OTS] * out;
  }
}

// Minibatch gradient, per-block partial sums.  Sample k of the batch is
// idx = (off + (b0 + k) * stride) mod n; the batch holds bsz samples (the
// loss is their mean).  Each block takes whole chunks of 64 samples; thread t
// owns gradient entries t, t + 256, ... (18 of them).
constexpr int GCH = 64;
constexpr int GPT = (NPAR + 255) / 256;

__global__ __launch_bounds__(256) void k_mlp_grad_partial(const float* __restrict__ model, const float* __restrict__ x,
                                                          const float* __restrict__ t, int64_t n, int64_t off,
                                                          int64_t stride, int64_t b0, int bsz,
                                                          float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ float w[NMODEL];
  __shared__ float xs[GCH][NIN];
  __shared__ float H1[GCH][NH], H2[GCH][NH], D2[GCH][NH], D1[GCH][NH];
  __shared__ float dout[GCH];
  __shared__ float lsum[GCH];
  const int tid = threadIdx.x;
  for (int e = tid; e < NMODEL; e += 256) w[e] = model[e];
  float acc[GPT];
#pragma unroll
  for (int q = 0; q < GPT; ++q) acc[q] = 0.f;
  float loss = 0.f;
  __syncthreads();
  const int nch = (bsz + GCH - 1) / GCH;
  for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    const int s0 = ch * GCH;
    const int cnt = (bsz - s0 < GCH) ? bsz - s0 : GCH;
    // inputs and standardized targets
    for (int e = tid; e < GCH * NIN; e += 256) {
      const int sl = e / NIN, k = e % NIN;
      float v = 0.f;
      if (sl < cnt) {
        const int64_t idx = (off + (b0 + s0 + sl) * stride) % n;
        v = (x[idx * NIN + k] - w[OXM + k]) / w[OXS + k];
      }
      xs[sl][k] = v;
    }
    __syncthreads();
    for (int e = tid; e < GCH * NH; e += 256) {
      const int sl = e / NH, j = e % NH;
      float a = w[OB1 + j];
      for (int k = 0; k < NIN; ++k) a += w[OW1 + j * NIN + k] * xs[sl][k];
      H1[sl][j] = tanhf(a);
    }
    __syncthreads();
    for (int e = tid; e < GCH * NH; e += 256) {
      const int sl = e / NH, j = e % NH;
      float a = w[OB2 + j];
      for (int k = 0; k < NH; ++k) a += w[OW2 + j * NH + k] * H1[sl][k];
      H2[sl][j] = tanhf(a);
    }
    __syncthreads();
    if (tid < GCH) {
      float o = w[OB3];
      for (int j = 0; j < NH; ++j) o += w[OW3 + j] * H2[tid][j];
      float r = 0.f;
      if (tid < cnt) {
        const int64_t idx = (off + (b0 + s0 + tid) * stride) % n;
        r = o - (t[idx] - w[OTM]) / w[OTS];
      }
      dout[tid] = 2.f * r / float(bsz);
      lsum[tid] = r * r / float(bsz);
    }
    __syncthreads();
    for (int e = tid; e < GCH * NH; e += 256) {
      const int sl = e / NH, j = e % NH;
      D2[sl][j] = dout[sl] * w[OW3 + j] * (1.f - H2[sl][j] * H2[sl][j]);
    }
    __syncthreads();
    for (int e = tid; e < GCH * NH; e += 256) {
      const int sl = e / NH, k = e % NH;
      float a = 0.f;
      for (int j = 0; j < NH; ++j) a += D2[sl][j] * w[OW2 + j * NH + k];
      D1[sl][k] = a * (1.f - H1[sl][k] * H1[sl][k]);
    }
    __syncthreads();
    if (tid == 0)
      for (int sl = 0; sl < GCH; ++sl) loss += lsum[sl];
#pragma unroll
    for (int q = 0; q < GPT; ++q) {
      const int e = tid + q * 256;
      if (e >= NPAR) continue;
      float g = 0.f;
      if (e < OB1) {
        const int j = (e - OW1) / NIN, k = (e - OW1) % NIN;
        for (int sl = 0; sl < GCH; ++sl) g += D1[sl][j] * xs[sl][k];
      } else if (e < OW2) {
        const int j = e - OB1;
        for (int sl = 0; sl < GCH; ++sl) g += D1[sl][j];
      } else if (e < OB2) {
        const int j = (e - OW2) / NH, k = (e - OW2) % NH;
        for (int sl = 0; sl < GCH; ++sl) g += D2[sl][j] * H1[sl][k];
      } else if (e < OW3) {
        const int j = e - OB2;
        for (int sl = 0; sl < GCH; ++sl) g += D2[sl][j];
      } else if (e < OB3) {
        const int j = e - OW3;
        for (int sl = 0; sl < GCH; ++sl) g += dout[sl] * H2[sl][j];
      } else {
        for (int sl = 0; sl < GCH; ++sl) g += dout[sl];
      }
      acc[q] += g;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < GPT; ++q) {
    const int e = tid + q * 256;
    if (e < NPAR) gpart[int64_t(blockIdx.x) * NPAR + e] = acc[q];
  }
  if (tid == 0) lpart[blockIdx.x] = loss;
}

// Sum of the block partials in block order: gradient and loss.
__global__ void k_mlp_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart, int nb,
                             float* __restrict__ grad, float* __restrict__ loss) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPAR; e += gridDim.x * blockDim.x) {
    float g = 0.f;
    for (int b = 0; b < nb; ++b) g += gpart[int64_t(b) * NPAR + e];
    grad[e] = g;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float l = 0.f;
    for (int b = 0; b < nb; ++b) l += lpart[b];
    loss[0] = l;
  }
}

// Adam on the summed partials; loss_acc[0] += batch loss.
__global__ void k_mlp_adam(const float* __restrict__ gpart, const float* __restrict__ lpart, int nb,
                           float* __restrict__ model, float* __restrict__ mom, float* __restrict__ vel, int step,
                           float lr, float b1, float b2, float eps, float* __restrict__ loss_acc) {
  const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPAR; e += gridDim.x * blockDim.x) {
    float g = 0.f;
    for (int b = 0; b < nb; ++b) g += gpart[int64_t(b) * NPAR + e];
    const float m = b1 * mom[e] + (1.f - b1) * g;
    const float v = b2 * vel[e] + (1.f - b2) * g * g;
    mom[e] = m;
    vel[e] = v;
    model[e] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss_acc) {
    float l = 0.f;
    for (int b = 0; b < nb; ++b) l += lpart[b];
    loss_acc[0] += l;
  }
}

// ---------------------------------------------------------------- budgeted selection
// Off-diagonal pair t is out of distribution when it lies beyond the training
// box on the side where pairs interact more: closer centroids than any
// training pair, larger overlaps, or spreads outside the training range
// (each widened by tol * span).  Pairs beyond the box on the far side
// (farther apart, smaller overlaps) are predicted with features clipped to
// the box, which over-estimates their contribution.
__global__ void k_ood_count(const float* __restrict__ f, int64_t np, int n, const float* __restrict__ model, float tol,
                            int* __restrict__ count) {
  int c = 0;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < np; t += int64_t(gridDim.x) * blockDim.x) {
    int i, j;
    tri_ij(t, n, i, j);
    if (i == j) continue;
    for (int k = 0; k < NIN; ++k) {
      const float lo = model[OXMIN + k], hi = model[OXMAX + k], span = hi - lo;
      const float v = f[t * NIN + k];
      const bool below = v < lo - tol * span, above = v > hi + tol * span;
      const bool risky = (k == 0) ? below : (k <= 2) ? (below || above) : above;
      if (risky) { ++c; break; }
    }
  }
  if (c) atomicAdd(count, c);
}

// Budget threshold preparation: q[t] = pred[t] for off-diagonal pairs and
// +inf for the diagonal (never dropped), w[t] = 10^pred[t] (0 on the diagonal).
__global__ void k_budget_prep(const float* __restrict__ pred, int64_t np, int n, float* __restrict__ q,
                              double* __restrict__ w) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < np; t += int64_t(gridDim.x) * blockDim.x) {
    int i, j;
    tri_ij(t, n, i, j);
    const double p = double(pred[t]);
    q[t] = (i == j) ? INFINITY : pred[t];
    w[t] = (i == j) ? 0.0 : pow(10.0, p);
  }
}

// Largest tau (in log10) with sum over off-diagonal pairs of 10^pred below
// tau at most budget; bisection in one workgroup over the prepared arrays.
__global__ __launch_bounds__(1024) void k_budget_threshold(const float* __restrict__ q, const double* __restrict__ w,
                                                           int64_t np, double budget, double* __restrict__ tau) {
  __shared__ double red[1024];
  __shared__ double lohi[2];
  // bracket: prediction range over the off-diagonal pairs
  double mn = 1e300, mx = -1e300;
  for (int64_t t = threadIdx.x; t < np; t += 1024) {
    const float v = q[t];
    if (v == INFINITY) continue;
    mn = fmin(mn, double(v));
    mx = fmax(mx, double(v));
  }
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) lohi[0] = red[0] - 1.0;
  __syncthreads();
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) lohi[1] = red[0] + 1.0;
  __syncthreads();
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lohi[0] + lohi[1]);
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < np; t += 1024)
      if (double(q[t]) < mid) s += w[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (red[0] <= budget) lohi[0] = mid; else lohi[1] = mid;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) tau[0] = lohi[0];
}

// keep[t] = diagonal, or off-diagonal with pred >= tau (learned rule), or
// O >= rho_cut (threshold rule when fallback is set).
__global__ void k_keep_flags(const float* __restrict__ pred, int64_t np, int n, const double* __restrict__ tau,
                             const double* __restrict__ O, double rho_cut, const int* __restrict__ fallback,
                             uint8_t* __restrict__ keep) {
  const bool fb = fallback && fallback[0] > 0;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < np; t += int64_t(gridDim.x) * blockDim.x) {
    int i, j;
    tri_ij(t, n, i, j);
    bool k;
    if (i == j) k = true;
    else if (fb) k = O[int64_t(i) * n + j] >= rho_cut;
    else k = double(pred[t]) >= tau[0];
    keep[t] = k ? 1 : 0;
  }
}

// Ordered compaction of kept pairs (triangle order = sorted by i, then j).
__global__ __launch_bounds__(1024) void k_compact_keep(const uint8_t* __restrict__ keep, int64_t np, int n,
                                                       int64_t cap, int32_t* __restrict__ pairs,
                                                       int64_t* __restrict__ count) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < np; c0 += blockDim.x) {
    const int64_t t = c0 + threadIdx.x;
    const bool k = t < np && keep[t];
    const unsigned long long bal = __ballot(k);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int64_t off = base;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    if (k) {
      const int64_t p = off + before;
      if (p < cap) {
        int i, j;
        tri_ij(t, n, i, j);
        pairs[2 * p] = i;
        pairs[2 * p + 1] = j;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t s = 0;
      for (int w = 0; w < int(blockDim.x / 64); ++w) s += wsum[w];
      base += s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = base;
}

// ---------------------------------------------------------------- launchers
static unsigned gridn(int64_t n, int nt, int cap = 4096) {
  int64_t g = (n + nt - 1) / nt;
  if (g > cap) g = cap;
  return unsigned(g < 1 ? 1 : g);
}

void launch_marginals(const double* phi, int norb, int n, double* pz, double* py, double* px, hipStream_t s) {
  hipLaunchKernelGGL(k_plane_marginals, dim3(n, norb), dim3(256), 0, s, phi, n, pz, py, px);
}
void launch_subsample(const double* phi, int norb, int n, int st, double* out, hipStream_t s) {
  const int m = n / st;
  hipLaunchKernelGGL(k_subsample, dim3(gridn(int64_t(norb) * m * m * m, 256)), dim3(256), 0, s, phi, norb, n, st, out);
}
void launch_centroids(const double* pz, const double* py, const double* px, int norb, int n, double L, double dV,
                      double* cen, double* spr, hipStream_t s) {
  hipLaunchKernelGGL(k_centroids, dim3(norb), dim3(256), 0, s, pz, py, px, n, L, dV, cen, spr);
}
void launch_pair_features(const int32_t* pairs, int64_t np, int norb, const double* cen, const double* spr,
                          const double* O, const double* P, double L, float* f, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_features, dim3(gridn(np, 256)), dim3(256), 0, s, pairs, np, norb, cen, spr, O, P, L, f);
}
void launch_mlp_init(float* m, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3(gridn(NMODEL, 256)), dim3(256), 0, s, m, seed);
}
int stats_blocks(int64_t n) { return int(gridn(n, 256, 256)); }
void launch_mlp_stats(const float* x, const float* t, int64_t n, double* part, float* m, hipStream_t s) {
  const int nb = stats_blocks(n);
  hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(256), 0, s, x, t, n, part);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(1), 0, s, part, nb, n, m);
}
void launch_mlp_forward(const float* m, const float* x, int64_t n, int clamp, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(gridn(n, 256, 2048)), dim3(256), 0, s, m, x, n, clamp, y);
}
int mlp_grad_blocks(int bsz) { return int(gridn(bsz, GCH, 1024)); }
void launch_mlp_grad_partial(const float* m, const float* x, const float* t, int64_t n, int64_t off, int64_t stride,
                             int64_t b0, int bsz, float* gpart, float* lpart, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3(mlp_grad_blocks(bsz)), dim3(256), 0, s, m, x, t, n, off, stride, b0,
                     bsz, gpart, lpart);
}
void launch_mlp_reduce(const float* gpart, const float* lpart, int nb, float* grad, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3(gridn(NPAR, 256)), dim3(256), 0, s, gpart, lpart, nb, grad, loss);
}
void launch_mlp_adam(const float* gpart, const float* lpart, int nb, float* m, float* mom, float* vel, int step,
                     float lr, float b1, float b2, float eps, float* loss_acc, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3(gridn(NPAR, 256)), dim3(256), 0, s, gpart, lpart, nb, m, mom, vel, step, lr, b1,
                     b2, eps, loss_acc);
}
void launch_select(const float* pred, const float* feats, int64_t np, int norb, const float* model, double budget,
                   const double* O, double rho_cut, float ood_tol, int* ood, double* tau, uint8_t* keep, int64_t cap,
                   int32_t* pairs, int64_t* count, float* q, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_ood_count, dim3(gridn(np, 256)), dim3(256), 0, s, feats, np, norb, model, ood_tol, ood);
  hipLaunchKernelGGL(k_budget_prep, dim3(gridn(np, 256)), dim3(256), 0, s, pred, np, norb, q, w);
  hipLaunchKernelGGL(k_budget_threshold, dim3(1), dim3(1024), 0, s, q, w, np, budget, tau);
  hipLaunchKernelGGL(k_keep_flags, dim3(gridn(np, 256)), dim3(256), 0, s, pred, np, norb, tau, O, rho_cut, ood, keep);
  hipLaunchKernelGGL(k_compact_keep, dim3(1), dim3(1024), 0, s, keep, np, norb, cap, pairs, count);
}

}  // namespace ace
