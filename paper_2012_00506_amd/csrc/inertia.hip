// Sylvester inertia of B - sigma I by band LDL^H without pivoting (FP64),
// one workgroup per shift.
//
// The live part of the factorisation at step k is the lower triangle of rows
// k .. k+b+1 (row k+b+1 still untouched, loaded during step k for use from
// step k+1).  It is kept in LDS by diagonals: diagonal d (entries A(c+d, c))
// is a circular buffer of L_d = b+2-d slots indexed by c mod L_d, which holds
// exactly its live columns k .. k+b+1-d, so the whole triangle takes
// (b+2)(b+3)/2 entries (136 KB at b = 128).  The slot freed by column k-1 of
// each diagonal receives the entering row's entry, which step k neither reads
// nor writes, so a single barrier per step suffices; k mod L_d is kept per
// diagonal in LDS, double-buffered by step parity.
#include "fb_internal.h"
#include "prof.h"

namespace fb {

static const int kInertiaThreads = 512;
static const size_t kLdsBudget = 160 * 1024;

__device__ __forceinline__ c128 band_entry(const c128* __restrict__ Bd, int64_t n,
                                           int64_t i, int64_t c, double sigma) {
  // A(i, c) = B(i, c) - sigma * delta_ic for 0 <= i - c <= b (caller checks)
  c128 v = gld(Bd + (i - c) * n + c);
  if (i == c) v.x -= sigma;
  return v;
}

static size_t inertia_lds_bytes(int b) {
  const size_t tri = (size_t)(b + 2) * (b + 3) / 2;
  return tri * sizeof(c128) + 3 * (size_t)(b + 2) * sizeof(int) + 64;
}

__global__ void __launch_bounds__(kInertiaThreads)
k_band_ldlh_inertia(const c128* __restrict__ Bd, int64_t n, int b,
                    const double* __restrict__ shifts, const double* __restrict__ stats,
                    int32_t* __restrict__ counts) {
  extern __shared__ __align__(16) char lds_raw[];
  const int M = b + 2;
  const int tri = M * (M + 1) / 2;
  c128* D = reinterpret_cast<c128*>(lds_raw);
  int* off = reinterpret_cast<int*>(D + tri);  // start of diagonal d
  int* kd = off + M;                           // [2][M]: k mod L_d, by step parity
  const int s = blockIdx.x;
  const double sigma = shifts[s];
  const double eps = 2.220446049250313e-16;
  const double pivmin = eps * eps * stats[0];
  const int t = threadIdx.x;

  for (int e = t; e < tri; e += blockDim.x) D[e] = mk(0.0, 0.0);
  for (int d = t; d < M; d += blockDim.x) {
    off[d] = d * M - d * (d - 1) / 2;
    kd[d] = 0;
    kd[M + d] = 0;
  }
  __syncthreads();
  // initial window: rows/columns 0 .. min(b, n-1)
  const int64_t top = (int64_t)b < n ? b : n - 1;
  for (int e = t; e < M * M; e += blockDim.x) {
    const int c = e / M, i = e % M;
    if (c <= i && i <= top && i - c <= b) D[off[i - c] + c] = band_entry(Bd, n, i, c, sigma);
  }
  // update mapping: columns jc = 1 + ucol of the trailing triangle, every
  // ugrps-th diagonal
  const int ucols = b, ugrps = kInertiaThreads / (b > 0 ? b : 1);
  const int ucol = t % ucols, ugrp = t / ucols;
  const int jc = ucol + 1;
  // entering row entries: diagonal d = t (<= b), fetched one step ahead
  c128 ent = mk(0.0, 0.0);
  auto fetch = [&](int64_t k) {
    const int64_t inew = k + b + 1;
    c128 v = mk(0.0, 0.0);
    if (t <= b && inew < n) v = band_entry(Bd, n, inew, inew - t, sigma);
    return v;
  };
  ent = fetch(0);
  __syncthreads();

  int neg = 0, zero = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int* kc = kd + (k & 1) * M;
    int* kn = kd + ((k & 1) ^ 1) * M;
    const c128 cur = ent;
    if (k + 1 < n) ent = fetch(k + 1);
    double dk = D[off[0] + kc[0]].x;
    if (fabs(dk) < pivmin) {
      ++zero;
      dk = -pivmin;
    } else if (dk < 0.0) {
      ++neg;
    }
    const int m = (int)((n - 1 - k) < b ? (n - 1 - k) : b);
    const double rdk = 1.0 / dk;
    // A(k+jc+d, k+jc) -= A(k+jc+d, k) conj(A(k+jc, k)) / d_k, 1 <= jc, jc+d <= m
    if (ugrp < ugrps && jc <= m) {
      const c128 ack = D[off[jc] + kc[jc]];
      const c128 ackr = mk(ack.x * rdk, -ack.y * rdk);  // conj(A(c,k)) / d_k
      for (int d = ugrp; d + jc <= m; d += ugrps) {
        const int ii = d + jc;
        const int L = M - d;
        int sl = kc[d] + jc;
        if (sl >= L) sl -= L;
        const c128 aik = D[off[ii] + kc[ii]];
        c128 v = D[off[d] + sl];
        v.x -= aik.x * ackr.x - aik.y * ackr.y;
        v.y -= aik.x * ackr.y + aik.y * ackr.x;
        D[off[d] + sl] = v;
      }
    }
    // entering row k+b+1 into the slot column k-1 left on every diagonal
    if (t <= b && k + b + 1 < n) {
      const int L = M - t;
      int sl = kc[t] - 1;
      if (sl < 0) sl += L;
      D[off[t] + sl] = cur;
    }
    if (t < M) {
      int v = kc[t] + 1;
      kn[t] = v >= M - t ? 0 : v;
    }
    __syncthreads();
  }
  if (t == 0) {
    counts[3 * s + 0] = neg;
    counts[3 * s + 1] = zero;
    counts[3 * s + 2] = (int32_t)(n - neg - zero);
  }
}

size_t inertia_scratch_bytes(const Band& bd, int nshift) {
  (void)bd;
  (void)nshift;
  return 0;  // the window always fits in LDS (b <= 128)
}

int launch_inertia(const Band& bd, int nshift, const double* shifts_dev, int32_t* cnt_dev,
                   void* scratch, hipStream_t st) {
  (void)scratch;
  if (nshift <= 0) return 0;
  const size_t smem = inertia_lds_bytes(bd.b);
  if (smem > kLdsBudget) return FB_ERR_INTERNAL;
  (void)hipFuncSetAttribute((const void*)k_band_ldlh_inertia,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  ProfScope ps(FB_PROF_INERTIA, st, 4.0 * (double)bd.n * bd.b * bd.b * nshift);
  k_band_ldlh_inertia<<<nshift, kInertiaThreads, smem, st>>>(bd.Bd, bd.n, bd.b, shifts_dev,
                                                               bd.stats, cnt_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
