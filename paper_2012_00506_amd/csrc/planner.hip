// Learned slice planner: band features (stochastic Chebyshev moments of the
// density of states, Section 3.1, plus cheap band statistics) and the
// 80 -> 256 -> 256 -> 64 network (BF16 MFMA operands, FP32 accumulation),
// its backward pass and Adam.
#include <math.h>

#include <algorithm>
#include <vector>

#include "planner.h"
#include "prof.h"
#include "solve_job.h"

namespace fb {

// ---------------------------------------------------------------- probes
// SplitMix64 mixing of a 64-bit counter (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double rademacher(uint64_t seed, int p, int64_t i) {
  uint64_t c = seed * (1ull << 40) + (uint64_t)p * (1ull << 32) + (uint64_t)i;
  return (splitmix64(c) & 1ull) ? -1.0 : 1.0;
}

// t_next = s ((B t_cur - c t_cur) / h) - t_prev (first step: s = 1, no
// t_prev; the zeroth: t = v); part[(p * nrb + rb)] = sum over the row block
// of v_i Re(t_next_i).
static const int kChRows = 256;
__global__ void __launch_bounds__(kChRows)
k_cheb_step(const c128* __restrict__ Bd, int64_t n, int b, double c, double h,
            const c128* __restrict__ tp, const c128* __restrict__ tc, c128* __restrict__ tn,
            int mode, uint64_t seed, double* __restrict__ part, int nrb) {
  const int p = blockIdx.y, rb = blockIdx.x, t = threadIdx.x;
  const int64_t i = (int64_t)rb * kChRows + t;
  __shared__ double red[kChRows];
  double dot = 0.0;
  if (i < n) {
    const double v = rademacher(seed, p, i);
    c128 out;
    if (mode == 0) {
      out = mk(v, 0.0);
    } else {
      const c128* x = tc + (int64_t)p * n;
      c128 acc = mk((Bd[i].x - c) * x[i].x, (Bd[i].x - c) * x[i].y);
      for (int d = 1; d <= b; ++d) {
        if (i - d >= 0) cmac(acc, Bd[(int64_t)d * n + i - d], x[i - d]);
        if (i + d < n) cmacc(acc, Bd[(int64_t)d * n + i], x[i + d]);
      }
      acc = mk(acc.x / h, acc.y / h);
      if (mode == 2) {
        c128 q = tp[(int64_t)p * n + i];
        acc = mk(2.0 * acc.x - q.x, 2.0 * acc.y - q.y);
      }
      out = acc;
    }
    tn[(int64_t)p * n + i] = out;
    dot = v * out.x;
  }
  red[t] = dot;
  __syncthreads();
  for (int s = kChRows / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) part[(size_t)p * nrb + rb] = red[0];
}

__global__ void k_cheb_collect(const double* __restrict__ part, int P, int nrb, int64_t n, int k,
                               int K, double* __restrict__ mu) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int rb = 0; rb < nrb; ++rb) s += part[(size_t)p * nrb + rb];
  mu[(size_t)p * (K + 1) + k] = s / (double)n;
}

// diagonal statistics: pass 0 -> [sum d, min d, max d, off-diagonal energy],
// pass 1 (mean known) -> [sum (d-m)^2, sum (d-m)^3, sum (d-m)^4]
__global__ void __launch_bounds__(256)
k_diag_stats(const c128* __restrict__ Bd, int64_t n, int b, int pass, const double* mean,
             double* __restrict__ part) {
  __shared__ double r0[256], r1[256], r2[256], r3[256];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = pass ? 0.0 : 1e308, a2 = pass ? 0.0 : -1e308, a3 = 0.0;
  const double m = pass ? *mean : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double d = Bd[i].x;
    if (pass == 0) {
      a0 += d;
      a1 = fmin(a1, d);
      a2 = fmax(a2, d);
      for (int k = 1; k <= b; ++k)
        if (i + k < n) a3 += 2.0 * cabs2(Bd[(int64_t)k * n + i]);
    } else {
      double e = d - m;
      a0 += e * e;
      a1 += e * e * e;
      a2 += e * e * e * e;
    }
  }
  r0[t] = a0;
  r1[t] = a1;
  r2[t] = a2;
  r3[t] = a3;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      r0[t] += r0[t + s];
      if (pass == 0) {
        r1[t] = fmin(r1[t], r1[t + s]);
        r2[t] = fmax(r2[t], r2[t + s]);
      } else {
        r1[t] += r1[t + s];
        r2[t] += r2[t + s];
      }
      r3[t] += r3[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[4 * blockIdx.x + 0] = r0[0];
    part[4 * blockIdx.x + 1] = r1[0];
    part[4 * blockIdx.x + 2] = r2[0];
    part[4 * blockIdx.x + 3] = r3[0];
  }
}

static const int kStatGrid = 64;

size_t features_workspace(const Band& bd, int P) {
  return (size_t)3 * bd.n * P * sizeof(c128) + 4096 + (size_t)P * ((bd.n + kChRows - 1) / kChRows) * 8 +
         (size_t)P * 32 * 8 + 4 * kStatGrid * 8 + 64;
}

// Chebyshev moments mu (host, P x (K+1)) of the ingested band
int cheb_moments_dev(const Band& bd, int K, int P, uint64_t seed, Arena& ar, double* mu_host,
                     double c, double h, hipStream_t st) {
  const int64_t n = bd.n;
  const int nrb = (int)((n + kChRows - 1) / kChRows);
  c128* t0 = ar.take<c128>((size_t)n * P);
  c128* t1 = ar.take<c128>((size_t)n * P);
  c128* t2 = ar.take<c128>((size_t)n * P);
  double* part = ar.take<double>((size_t)P * nrb);
  double* mu = ar.take<double>((size_t)P * (K + 1));
  if (ar.base == nullptr) return 0;
  if (!ar.fits()) return FB_ERR_NOMEM;
  dim3 grid(nrb, P);
  c128 *a = t0, *bcur = t1, *nxt = t2;
  for (int k = 0; k <= K; ++k) {
    int mode = k == 0 ? 0 : (k == 1 ? 1 : 2);
    // k = 0: a <- v;  k = 1: bcur <- Bh a;  k >= 2: nxt <- 2 Bh bcur - a
    c128* out = k == 0 ? a : (k == 1 ? bcur : nxt);
    const c128* cur = k == 1 ? a : bcur;
    const c128* prev = a;
    k_cheb_step<<<grid, kChRows, 0, st>>>(bd.Bd, n, bd.b, c, h, prev, cur, out, mode, seed, part,
                                          nrb);
    FB_HIP(hipGetLastError());
    k_cheb_collect<<<(P + 63) / 64, 64, 0, st>>>(part, P, nrb, n, k, K, mu);
    FB_HIP(hipGetLastError());
    if (k >= 2) {  // rotate: (a, bcur, nxt) <- (bcur, nxt, a)
      c128* tmp = a;
      a = bcur;
      bcur = nxt;
      nxt = tmp;
    }
  }
  FB_HIP(hipMemcpyAsync(mu_host, mu, sizeof(double) * P * (K + 1), hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  return 0;
}

static double jackson(int k, int K) {
  const double N = K + 1, a = M_PI / (N + 1);
  return ((N - k + 1) * cos(a * k) + sin(a * k) / tan(a)) / (N + 1);
}

int band_features_dev(const Band& bd, uint64_t seed, Arena& ar, double* feat, hipStream_t st) {
  const int K = kPlanK, P = kPlanP;
  double* part = ar.take<double>(4 * kStatGrid);
  double* dmean = ar.take<double>(1);
  std::vector<double> mu((size_t)P * (K + 1));
  double stats[3] = {0, 0, 0};
  if (ar.base) FB_TRY(band_stats_host(bd, stats, st));
  const double nrm = stats[0], lo = stats[1], hi = stats[2];
  const double c = 0.5 * (lo + hi), h = 1.01 * 0.5 * (hi - lo);
  FB_TRY(cheb_moments_dev(bd, K, P, seed, ar, mu.data(), c, h, st));
  if (ar.base == nullptr) return 0;
  // diagonal statistics
  double p0[4 * kStatGrid], p1[4 * kStatGrid];
  k_diag_stats<<<kStatGrid, 256, 0, st>>>(bd.Bd, bd.n, bd.b, 0, nullptr, part);
  FB_HIP(hipGetLastError());
  FB_HIP(hipMemcpyAsync(p0, part, sizeof p0, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  double sum = 0, mn = 1e308, mx = -1e308, off = 0;
  for (int g = 0; g < kStatGrid; ++g) {
    sum += p0[4 * g];
    mn = std::min(mn, p0[4 * g + 1]);
    mx = std::max(mx, p0[4 * g + 2]);
    off += p0[4 * g + 3];
  }
  const double n = (double)bd.n, mean = sum / n;
  FB_HIP(hipMemcpyAsync(dmean, &mean, sizeof(double), hipMemcpyHostToDevice, st));
  k_diag_stats<<<kStatGrid, 256, 0, st>>>(bd.Bd, bd.n, bd.b, 1, dmean, part);
  FB_HIP(hipGetLastError());
  FB_HIP(hipMemcpyAsync(p1, part, sizeof p1, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  double m2 = 0, m3 = 0, m4 = 0;
  for (int g = 0; g < kStatGrid; ++g) {
    m2 += p1[4 * g];
    m3 += p1[4 * g + 1];
    m4 += p1[4 * g + 2];
  }
  m2 /= n;
  m3 /= n;
  m4 /= n;
  const double sd = sqrt(m2);
  const double skew = sd > 0 ? m3 / (sd * sd * sd) : 0.0;
  const double kurt = sd > 0 ? m4 / (m2 * m2) - 3.0 : 0.0;
  // assemble the 80 features
  int f = 0;
  feat[f++] = lo / nrm;
  feat[f++] = hi / nrm;
  std::vector<double> mbar(K + 1, 0.0), msd(K + 1, 0.0);
  for (int k = 0; k <= K; ++k) {
    for (int p = 0; p < P; ++p) mbar[k] += mu[(size_t)p * (K + 1) + k];
    mbar[k] /= P;
    for (int p = 0; p < P; ++p) {
      double e = mu[(size_t)p * (K + 1) + k] - mbar[k];
      msd[k] += e * e;
    }
    msd[k] = sqrt(msd[k] / P);
  }
  for (int k = 1; k <= K; ++k) feat[f++] = mbar[k];
  for (int k = 1; k <= K; ++k) feat[f++] = msd[k];
  for (int i = 0; i < 32; ++i) {
    double t = lo + (i + 0.5) * (hi - lo) / 32.0;
    double th = acos(std::min(1.0, std::max(-1.0, (t - c) / h)));
    double val = jackson(0, K) * mbar[0] * (M_PI - th);
    for (int k = 1; k <= K; ++k) val -= 2.0 * jackson(k, K) * mbar[k] * sin(k * th) / k;
    feat[f++] = val / M_PI;
  }
  const double fro2 = m2 * n + mean * mean * n + off;
  feat[f++] = log2(n) / 16.0;
  feat[f++] = bd.b0 / 128.0;
  feat[f++] = bd.cplx ? 1.0 : 0.0;
  feat[f++] = mean / nrm;
  feat[f++] = sd / nrm;
  feat[f++] = mn / nrm;
  feat[f++] = mx / nrm;
  feat[f++] = skew;
  feat[f++] = kurt / 10.0;
  feat[f++] = off / n / (nrm * nrm);
  feat[f++] = log10(nrm);
  feat[f++] = (hi - lo) / nrm;
  feat[f++] = fro2 / n / (nrm * nrm);
  feat[f++] = (mx - mn) / (hi - lo);
  return f == kPlanFeatures ? 0 : FB_ERR_INTERNAL;
}

// ---------------------------------------------------------------- network
typedef float pl_f4 __attribute__((ext_vector_type(4)));
typedef short pl_s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
  // round to nearest, ties to even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C[M x N] = op(A) op(B) (+ bias[col]) with epilogue: ReLU, or multiply by
// (mask > 0), or add-to; operands read as FP32 and rounded to BF16, MFMA
// 16x16x16 with FP32 accumulation.  Element (i, k) of op(A) is
// A[i * sai + k * sak], (k, j) of op(B) is B[k * sbk + j * sbj].
// One wave per 16 x 16 tile of C.
struct GemmArgs {
  int M, N, K;
  const float* A;
  int sai, sak;
  const float* B;
  int sbk, sbj;
  float* C;
  int ldc;
  const float* bias;  // per column, or null
  const float* mask;  // C *= (mask > 0) elementwise (ld = ldc), or null
  int relu;
};

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tiles_n = (g.N + 15) / 16;
  const int tile = blockIdx.x * 4 + wv;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  if (tm * 16 >= g.M) return;
  const int i = tm * 16 + (lane & 15), j = tn * 16 + (lane & 15), kq = 4 * (lane >> 4);
  pl_f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    pl_s4 a, b;
    for (int v = 0; v < 4; ++v) {
      int k = k0 + kq + v;
      float av = (i < g.M && k < g.K) ? g.A[(size_t)i * g.sai + (size_t)k * g.sak] : 0.f;
      float bv = (j < g.N && k < g.K) ? g.B[(size_t)k * g.sbk + (size_t)j * g.sbj] : 0.f;
      a[v] = to_bf16(av);
      b[v] = to_bf16(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  for (int r = 0; r < 4; ++r) {
    int row = tm * 16 + 4 * (lane >> 4) + r, col = tn * 16 + (lane & 15);
    if (row >= g.M || col >= g.N) continue;
    float v = acc[r];
    if (g.bias) v += g.bias[col];
    if (g.relu) v = fmaxf(v, 0.f);
    if (g.mask && !(g.mask[(size_t)row * g.ldc + col] > 0.f)) v = 0.f;
    g.C[(size_t)row * g.ldc + col] = v;
  }
}

static int gemm(const GemmArgs& g, hipStream_t st) {
  int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
  k_gemm_bf16<<<(tiles + 3) / 4, 256, 0, st>>>(g);
  FB_HIP(hipGetLastError());
  return 0;
}

// dY = 2 (Y - T) / (B * 64); loss partials
__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T,
                           float* __restrict__ dY, int count, float scale,
                           float* __restrict__ lpart) {
  __shared__ float red[256];
  float s = 0.f;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
    float d = Y[e] - T[e];
    dY[e] = 2.f * d * scale;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// column sums of a rows x cols row-major array (bias gradients)
__global__ void k_colsum(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
  out[c] = s;
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
    float gg = g[e];
    float mm = b1 * m[e] + (1.f - b1) * gg;
    float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

__global__ void k_lossfinal(const float* __restrict__ lpart, int nb, float inv, float* __restrict__ loss) {
  if (threadIdx.x || blockIdx.x) return;
  float s = 0.f;
  for (int i = 0; i < nb; ++i) s += lpart[i];
  *loss = s * inv;
}

struct Net {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static Net net_of(const float* w) {
  Net n;
  n.W1 = w;
  n.b1 = n.W1 + kH0 * kH1;
  n.W2 = n.b1 + kH1;
  n.b2 = n.W2 + kH1 * kH2;
  n.W3 = n.b2 + kH2;
  n.b3 = n.W3 + kH2 * kH3;
  return n;
}

size_t net_scratch_floats(int batch) { return (size_t)batch * (2 * kH1 + 2 * kH2 + 3 * kH3) + 1024; }

int net_forward(const float* w, int batch, const float* X, float* Y, float* H1, float* H2,
                hipStream_t st) {
  Net n = net_of(w);
  FB_TRY(gemm({batch, kH1, kH0, X, kH0, 1, n.W1, kH1, 1, H1, kH1, n.b1, nullptr, 1}, st));
  FB_TRY(gemm({batch, kH2, kH1, H1, kH1, 1, n.W2, kH2, 1, H2, kH2, n.b2, nullptr, 1}, st));
  FB_TRY(gemm({batch, kH3, kH2, H2, kH2, 1, n.W3, kH3, 1, Y, kH3, n.b3, nullptr, 0}, st));
  return 0;
}

}  // namespace fb

using namespace fb;

extern "C" size_t fb_planner_bytes(void) { return sizeof(float) * (size_t)kNetParams; }

extern "C" int band_features(const fb_band* B, uint64_t seed, double* feat, void* work,
                             size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (!feat) return -3;
  if (!lwork) return -5;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  bd.b0 = B->b;
  FB_TRY(band_features_dev(bd, seed, ar, feat, st));
  if (work == nullptr) *lwork = ar.used;
  return 0;
}

extern "C" int band_cheb_moments(const fb_band* B, int32_t K, int32_t P, uint64_t seed, double* mu,
                                 double* gersh, void* work, size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (K < 0 || K > 1000) return -2;
  if (P < 1 || P > 4096) return -3;
  if (!mu) return -5;
  if (!lwork) return -8;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  double stats[3] = {0, 0, 0};
  if (ar.base) FB_TRY(band_stats_host(bd, stats, st));
  const double c = 0.5 * (stats[1] + stats[2]), h = 1.01 * 0.5 * (stats[2] - stats[1]);
  FB_TRY(cheb_moments_dev(bd, K, P, seed, ar, mu, c, h, st));
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (gersh) {
    gersh[0] = stats[1];
    gersh[1] = stats[2];
    gersh[2] = stats[0];
  }
  return 0;
}

extern "C" int planner_forward(const void* weights, int32_t batch, const float* x, float* out,
                               void* work, size_t* lwork, void* stream) {
  if (!weights) return -1;
  if (batch < 1) return -2;
  if (!x) return -3;
  if (!out) return -4;
  if (!lwork) return -6;
  size_t need = sizeof(float) * (size_t)batch * (kH1 + kH2) + 512;
  if (!work) {
    *lwork = need;
    return 0;
  }
  if (*lwork < need) return FB_ERR_NOMEM;
  float* H1 = (float*)work;
  float* H2 = H1 + (size_t)batch * kH1;
  return net_forward((const float*)weights, batch, x, out, H1, H2, (hipStream_t)stream);
}

extern "C" int planner_train_step(void* weights, void* opt_state, int32_t batch, const float* x,
                                  const float* target, float lr, int32_t t, float* loss,
                                  void* grads, void* work, size_t* lwork, void* stream) {
  if (!weights) return -1;
  if (!opt_state && !grads) return -2;
  if (batch < 1) return -3;
  if (!x) return -4;
  if (!target) return -5;
  if (!(lr >= 0.f)) return -6;
  if (t < 1 && !grads) return -7;
  if (!lwork) return -11;
  const size_t nf = (size_t)batch;
  size_t need = sizeof(float) * (nf * (2 * kH1 + 2 * kH2 + 2 * kH3) + (size_t)kNetParams + 1024);
  if (!work) {
    *lwork = need;
    return 0;
  }
  if (*lwork < need) return FB_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  float* w = (float*)weights;
  Net n = net_of(w);
  float* H1 = (float*)work;
  float* H2 = H1 + nf * kH1;
  float* Y = H2 + nf * kH2;
  float* dY = Y + nf * kH3;
  float* dZ2 = dY + nf * kH3;
  float* dZ1 = dZ2 + nf * kH2;
  float* G = grads ? (float*)grads : dZ1 + nf * kH1;
  float* lpart = G + kNetParams;
  float* ldev = lpart + 256;
  float *gW1 = G, *gb1 = gW1 + kH0 * kH1, *gW2 = gb1 + kH1, *gb2 = gW2 + kH1 * kH2,
        *gW3 = gb2 + kH2, *gb3 = gW3 + kH2 * kH3;
  FB_TRY(net_forward(w, batch, x, Y, H1, H2, st));
  const int cnt = batch * kH3;
  const int lb = std::min(256, (cnt + 255) / 256);
  k_mse_grad<<<lb, 256, 0, st>>>(Y, target, dY, cnt, 1.f / (float)cnt, lpart);
  FB_HIP(hipGetLastError());
  // W3: H2^T dY, b3: colsum dY, dZ2 = (dY W3^T) * (H2 > 0)
  FB_TRY(gemm({kH2, kH3, batch, H2, 1, kH2, dY, kH3, 1, gW3, kH3, nullptr, nullptr, 0}, st));
  k_colsum<<<(kH3 + 63) / 64, 64, 0, st>>>(dY, batch, kH3, gb3);
  FB_TRY(gemm({batch, kH2, kH3, dY, kH3, 1, n.W3, 1, kH3, dZ2, kH2, nullptr, H2, 0}, st));
  FB_TRY(gemm({kH1, kH2, batch, H1, 1, kH1, dZ2, kH2, 1, gW2, kH2, nullptr, nullptr, 0}, st));
  k_colsum<<<(kH2 + 63) / 64, 64, 0, st>>>(dZ2, batch, kH2, gb2);
  FB_TRY(gemm({batch, kH1, kH2, dZ2, kH2, 1, n.W2, 1, kH2, dZ1, kH1, nullptr, H1, 0}, st));
  FB_TRY(gemm({kH0, kH1, batch, x, 1, kH0, dZ1, kH1, 1, gW1, kH1, nullptr, nullptr, 0}, st));
  k_colsum<<<(kH1 + 63) / 64, 64, 0, st>>>(dZ1, batch, kH1, gb1);
  FB_HIP(hipGetLastError());
  k_lossfinal<<<1, 1, 0, st>>>(lpart, lb, 1.f / (float)cnt, ldev);
  FB_HIP(hipGetLastError());
  if (!grads) {
    float* m = (float*)opt_state;
    float* v = m + kNetParams;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_adam<<<256, 256, 0, st>>>(w, m, v, G, kNetParams, lr, b1, b2, 1e-8f, c1, c2);
    FB_HIP(hipGetLastError());
  }
  if (loss) {
    FB_HIP(hipMemcpyAsync(loss, ldev, sizeof(float), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
  }
  return 0;
}
