// Blocked Cholesky factorisation G = R^H R and triangular inverse T = R^{-1}
// of a batch of Hermitian positive definite matrices (complex128), for the
// Cholesky QR orthonormalisation of the filtered block (Algorithm alg:FEAST).
//
// Block columns of 64: the diagonal block is factored (and its triangular
// inverse formed) by one workgroup in LDS; the row panel R(k, k+1:) =
// R(k,k)^{-H} G(k, k+1:) and the trailing update G(k+1:, k+1:) -=
// R(k, k+1:)^H R(k, k+1:) are batched FP64-MFMA products (gemm64).  The
// inverse follows by block columns, T(0:j, j) = -T(0:j, 0:j) R(0:j, j)
// R(j, j)^{-1}.  Every matrix of the batch advances in the same launches.
#include <math.h>

#include <algorithm>

#include "chol64.h"
#include "prof.h"

namespace fb {

namespace {
constexpr int BS = 64;
constexpr int LDS_LD = BS + 1;  // padded column length of the LDS block
}  // namespace

// Factor the diagonal block kb of every matrix: R(k,k) (upper, zero below
// the diagonal) back into G, its inverse into Dinv + kb * 64 * 64 (ld 64,
// zero-padded).  A pivot r_jj^2 not above piv_min (or NaN) records the
// 1-based column in *info (first failure only) and is replaced by 1 so
// that the rest of the batch stays finite.
__global__ void __launch_bounds__(256)
k_chol_diag(const CholProb* __restrict__ probs, int kb, double piv_min) {
  extern __shared__ __align__(16) char lds_raw[];
  c128* S = reinterpret_cast<c128*>(lds_raw);  // column-major: S[j * LDS_LD + i] = block(i, j)
  c128* U = S + BS * LDS_LD;                   // the inverse
  __shared__ int fail;
  const CholProb P = probs[blockIdx.x];
  const int nblk = (P.m + BS - 1) / BS;
  if (kb >= nblk) return;
  const int k0 = kb * BS, bs = min(BS, P.m - k0);
  const int t = threadIdx.x;
  if (t == 0) fail = 0;
  for (int e = t; e < BS * BS; e += blockDim.x) {
    const int j = e / BS, i = e % BS;
    c128 v = mk(0.0, 0.0);
    if (i <= j && j < bs) v = gld(P.G + (int64_t)(k0 + j) * P.ld + k0 + i);
    S[j * LDS_LD + i] = v;
    U[j * LDS_LD + i] = mk(0.0, 0.0);
  }
  __syncthreads();
  // right-looking Cholesky on the upper triangle
  for (int j = 0; j < bs; ++j) {
    double d = S[j * LDS_LD + j].x;
    if (!(d > piv_min)) {
      if (t == 0 && fail == 0) fail = k0 + j + 1;
      d = 1.0;
    }
    const double r = sqrt(d), ri = 1.0 / r;
    __syncthreads();  // everyone has read the pivot
    for (int k = j + t; k < bs; k += blockDim.x)
      S[k * LDS_LD + j] = k == j ? mk(r, 0.0) : ri * S[k * LDS_LD + j];
    __syncthreads();
    // S(i, k) -= conj(S(j, i)) S(j, k), j < i <= k
    const int rem = bs - j - 1;
    for (int e = t; e < rem * rem; e += blockDim.x) {
      const int i = j + 1 + e % rem, k = j + 1 + e / rem;
      if (i > k) continue;
      c128 v = S[k * LDS_LD + i];
      cmacc(v, mk(-S[i * LDS_LD + j].x, -S[i * LDS_LD + j].y), S[k * LDS_LD + j]);
      S[k * LDS_LD + i] = v;
    }
    __syncthreads();
  }
  // inverse by columns: U(j,j) = 1/R(j,j); U(i,j) = -(sum_{l=i}^{j-1} U(i,l) R(l,j)) / R(j,j)
  for (int j = 0; j < bs; ++j) {
    const double rjj = S[j * LDS_LD + j].x;
    for (int i = t; i <= j; i += blockDim.x) {
      if (i == j) {
        U[j * LDS_LD + j] = mk(1.0 / rjj, 0.0);
      } else {
        c128 acc = mk(0.0, 0.0);
        for (int l = i; l < j; ++l) cmac(acc, U[l * LDS_LD + i], S[j * LDS_LD + l]);
        U[j * LDS_LD + i] = (-1.0 / rjj) * acc;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < BS * BS; e += blockDim.x) {
    const int j = e / BS, i = e % BS;
    if (i < bs && j < bs) gst(P.G + (int64_t)(k0 + j) * P.ld + k0 + i, S[j * LDS_LD + i]);
    gst(P.Dinv + (size_t)kb * BS * BS + (size_t)j * BS + i, U[j * LDS_LD + i]);
  }
  // the first block starts the record; later blocks keep the first failure
  if (t == 0 && (kb == 0 || (fail && gld(P.info) == 0))) gst(P.info, fail);
}

// T = 0 with the diagonal blocks set to Dinv
__global__ void __launch_bounds__(256) k_tri_init(const CholProb* __restrict__ probs) {
  const CholProb P = probs[blockIdx.y];
  const int m = P.m;
  const int64_t tot = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    c128 v = mk(0.0, 0.0);
    if (i / BS == j / BS)
      v = gld(P.Dinv + (size_t)(j / BS) * BS * BS + (size_t)(j % BS) * BS + i % BS);
    gst(P.T + (int64_t)j * P.ldt + i, v);
  }
}

// T(i, :) *= rowscale(i)
__global__ void __launch_bounds__(256) k_tri_rowscale(const CholProb* __restrict__ probs) {
  const CholProb P = probs[blockIdx.y];
  if (!P.rowscale) return;
  const int m = P.m;
  const int64_t tot = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    if (i > j) continue;
    c128* p = P.T + (int64_t)j * P.ldt + i;
    gst(p, gld(P.rowscale + i) * gld(p));
  }
}

size_t chol_gemm_descs(int nprob, int m_max) {
  const int nblk = (m_max + BS - 1) / BS;
  return (size_t)nprob * (2 * (size_t)nblk + 2 * (size_t)nblk);
}

int chol_inverse(const std::vector<CholProb>& probs, CholProb* probs_dev, GemmProb* gdev,
                 size_t gcap, double piv_min, hipStream_t st) {
  const int np = (int)probs.size();
  if (np == 0) return 0;
  int nblk = 0;
  for (const CholProb& p : probs) nblk = std::max(nblk, (p.m + BS - 1) / BS);
  // every product of every step, copied to the device once
  std::vector<GemmProb> g;
  std::vector<std::pair<size_t, GemmBatch>> steps;
  auto add_step = [&](auto fill) -> int {
    const size_t off = g.size();
    for (int q = 0; q < np; ++q) g.push_back(fill(probs[q]));
    GemmBatch b;
    FB_TRY(gemm_prepare(g.data() + off, np, b));
    steps.push_back({off, b});
    return 0;
  };
  auto base = [](const CholProb&) {
    GemmProb p{};
    p.alpha = mk(1.0, 0.0);
    p.ksplit = 1;
    return p;
  };
  for (int kb = 0; kb < nblk; ++kb) {
    // row panel: R(k, k+1:) = Dinv_k^H G(k, k+1:), in place
    FB_TRY(add_step([&](const CholProb& c) {
      GemmProb p = base(c);
      const int k0 = kb * BS, bs = std::min(BS, c.m - k0), rest = c.m - k0 - BS;
      if (bs <= 0 || rest <= 0) return p;  // M = N = 0: no work
      p.transa = 1;
      p.A = c.Dinv + (size_t)kb * BS * BS;
      p.lda = BS;
      p.B = c.G + (int64_t)(k0 + BS) * c.ld + k0;
      p.ldb = c.ld;
      p.C = c.G + (int64_t)(k0 + BS) * c.ld + k0;
      p.ldc = c.ld;
      p.M = bs;
      p.N = rest;
      p.K = bs;
      return p;
    }));
    // trailing update of the upper triangle: G(k+1:, k+1:) -= R(k, k+1:)^H R(k, k+1:)
    FB_TRY(add_step([&](const CholProb& c) {
      GemmProb p = base(c);
      const int k0 = kb * BS, bs = std::min(BS, c.m - k0), rest = c.m - k0 - BS;
      if (bs <= 0 || rest <= 0) return p;
      p.transa = 1;
      p.herm = 1;
      p.A = c.G + (int64_t)(k0 + BS) * c.ld + k0;
      p.lda = c.ld;
      p.B = p.A;
      p.ldb = c.ld;
      p.C = c.G + (int64_t)(k0 + BS) * c.ld + k0 + BS;
      p.ldc = c.ld;
      p.M = p.N = rest;
      p.K = bs;
      p.alpha = mk(-1.0, 0.0);
      p.beta = 1;
      return p;
    }));
  }
  for (int jb = 1; jb < nblk; ++jb) {
    // P = R(0:j, j) Dinv_j
    FB_TRY(add_step([&](const CholProb& c) {
      GemmProb p = base(c);
      const int j0 = jb * BS, bs = std::min(BS, c.m - j0);
      if (bs <= 0) return p;
      p.A = c.G + (int64_t)j0 * c.ld;
      p.lda = c.ld;
      p.B = c.Dinv + (size_t)jb * BS * BS;
      p.ldb = BS;
      p.C = c.P;
      p.ldc = c.m;
      p.M = j0;
      p.N = bs;
      p.K = bs;
      return p;
    }));
    // T(0:j, j) = -T(0:j, 0:j) P
    FB_TRY(add_step([&](const CholProb& c) {
      GemmProb p = base(c);
      const int j0 = jb * BS, bs = std::min(BS, c.m - j0);
      if (bs <= 0) return p;
      p.A = c.T;
      p.lda = c.ldt;
      p.a_upper = 1;
      p.B = c.P;
      p.ldb = c.m;
      p.C = c.T + (int64_t)j0 * c.ldt;
      p.ldc = c.ldt;
      p.M = j0;
      p.N = bs;
      p.K = j0;
      p.alpha = mk(-1.0, 0.0);
      return p;
    }));
  }
  if (g.size() > gcap) return FB_ERR_INTERNAL;
  FB_HIP(hipMemcpyAsync(probs_dev, probs.data(), sizeof(CholProb) * np, hipMemcpyHostToDevice, st));
  if (!g.empty())
    FB_HIP(hipMemcpyAsync(gdev, g.data(), sizeof(GemmProb) * g.size(), hipMemcpyHostToDevice, st));
  const size_t dlds = 2 * (size_t)BS * LDS_LD * sizeof(c128);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_chol_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)dlds);
    (void)hipGetLastError();
    attr = true;
  }
  size_t si = 0;
  for (int kb = 0; kb < nblk; ++kb) {
    k_chol_diag<<<np, 256, dlds, st>>>(probs_dev, kb, piv_min);
    FB_HIP(hipGetLastError());
    for (int r = 0; r < 2; ++r, ++si) FB_TRY(gemm_launch(gdev + steps[si].first, steps[si].second, st));
  }
  int mmax = 0;
  for (const CholProb& p : probs) mmax = std::max(mmax, p.m);
  const int grid = (int)std::min<int64_t>(((int64_t)mmax * mmax + 255) / 256, 4096);
  k_tri_init<<<dim3(grid, np), 256, 0, st>>>(probs_dev);
  FB_HIP(hipGetLastError());
  for (; si < steps.size(); ++si) FB_TRY(gemm_launch(gdev + steps[si].first, steps[si].second, st));
  k_tri_rowscale<<<dim3(grid, np), 256, 0, st>>>(probs_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
