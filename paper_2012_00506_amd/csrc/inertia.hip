// Sylvester inertia of B - sigma I by band LDL^H without pivoting (FP64),
// one workgroup per shift.
//
// The live part of the factorisation at step k is the lower triangle of the
// rows/columns k .. k+b of the partially reduced matrix.  Row k+b+1 (still
// untouched by the elimination) is loaded during step k for use at step k+1.
// Both are kept in an M x M circular window, M = b + 2, slot
// (c mod M, i mod M) holding A(i, c) for c <= i: every live entry has a
// distinct slot, the entering row (row slot (k-1) mod M) is neither read nor
// written by step k, and a single barrier per step suffices.  The window sits in LDS when it fits and
// in a per-shift global scratch area otherwise.
#include "fb_internal.h"
#include "prof.h"

namespace fb {

static const int kInertiaThreads = 256;
static const size_t kLdsBudget = 160 * 1024;

__device__ __forceinline__ c128 band_entry(const c128* __restrict__ Bd, int64_t n,
                                           int64_t i, int64_t c, double sigma) {
  // A(i, c) = B(i, c) - sigma * delta_ic for 0 <= i - c <= b (caller checks)
  c128 v = Bd[(i - c) * n + c];
  if (i == c) v.x -= sigma;
  return v;
}

template <bool USE_LDS>
__global__ void __launch_bounds__(kInertiaThreads)
k_band_ldlh_inertia(const c128* __restrict__ Bd, int64_t n, int b,
                    const double* __restrict__ shifts, const double* __restrict__ stats,
                    int32_t* __restrict__ counts, c128* __restrict__ gwin) {
  extern __shared__ c128 lds_win[];
  const int M = b + 2;
  const int s = blockIdx.x;
  // the LDS window is a compile-time choice, so that its accesses are LDS
  // instructions rather than flat ones
  c128* W = USE_LDS ? lds_win : gwin + (size_t)s * M * M;
  const double sigma = shifts[s];
  const double eps = 2.220446049250313e-16;
  const double pivmin = eps * eps * stats[0];
  const int t = threadIdx.x;

  // initial window: rows/columns 0 .. min(b, n-1)
  int64_t top = (int64_t)b < n ? b : n - 1;
  for (int idx = t; idx < M * M; idx += blockDim.x) {
    int cs = idx / M, rs = idx % M;
    int64_t c = cs, i = rs;
    c128 v = mk(0.0, 0.0);
    if (c <= i && i <= top && i - c <= b) v = band_entry(Bd, n, i, c, sigma);
    W[cs * M + rs] = v;
  }
  __syncthreads();

  int neg = 0, zero = 0;
  int ks = 0;  // k mod M; offsets below M need at most one wrap
  auto slot = [&](int off) { int v = ks + off; return v >= M ? v - M : v; };
  for (int64_t k = 0; k < n; ++k) {
    double dk = W[ks * M + ks].x;
    if (fabs(dk) < pivmin) {
      ++zero;
      dk = -pivmin;
    } else if (dk < 0.0) {
      ++neg;
    }
    const int m = (int)((n - 1 - k) < b ? (n - 1 - k) : b);
    const double rdk = 1.0 / dk;
    // rank-one update of the trailing triangle: for k < c <= i <= k+m
    // A(i, c) -= A(i, k) conj(A(c, k)) / d_k
    for (int idx = t; idx < m * m; idx += blockDim.x) {
      int ii = idx / m + 1;  // i - k
      int jc = idx - (ii - 1) * m + 1;  // c - k
      if (jc > ii) continue;
      int is = slot(ii), cs = slot(jc);
      c128 aik = W[ks * M + is];
      c128 ack = W[ks * M + cs];
      c128 upd = W[cs * M + is];
      c128 p = aik * cconj(ack);
      upd.x -= p.x * rdk;
      upd.y -= p.y * rdk;
      W[cs * M + is] = upd;
    }
    // entering row i = k+b+1 (columns k+1 .. k+b+1), used from step k+1 on
    int64_t inew = k + b + 1;
    if (inew < n) {
      const int rs = slot(b + 1);
      for (int jc = t; jc <= b; jc += blockDim.x) {
        int64_t c = inew - b + jc;  // columns inew-b .. inew
        W[slot(1 + jc) * M + rs] = band_entry(Bd, n, inew, c, sigma);
      }
    }
    __syncthreads();
    ks = slot(1);
  }
  if (t == 0) {
    counts[3 * s + 0] = neg;
    counts[3 * s + 1] = zero;
    counts[3 * s + 2] = (int32_t)(n - neg - zero);
  }
}

static bool inertia_lds(int b) { return (size_t)(b + 2) * (b + 2) * sizeof(c128) <= kLdsBudget; }

size_t inertia_scratch_bytes(const Band& bd, int nshift) {
  if (inertia_lds(bd.b)) return 0;
  return (size_t)nshift * (bd.b + 2) * (bd.b + 2) * sizeof(c128);
}

int launch_inertia(const Band& bd, int nshift, const double* shifts_dev, int32_t* cnt_dev,
                   void* scratch, hipStream_t st) {
  if (nshift <= 0) return 0;
  bool lds = inertia_lds(bd.b);
  size_t smem = lds ? (size_t)(bd.b + 2) * (bd.b + 2) * sizeof(c128) : 0;
  if (lds) {
    (void)hipFuncSetAttribute((const void*)k_band_ldlh_inertia<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    (void)hipGetLastError();
  }
  ProfScope ps(FB_PROF_INERTIA, st, 4.0 * (double)bd.n * bd.b * bd.b * nshift);
  if (lds)
    k_band_ldlh_inertia<true><<<nshift, kInertiaThreads, smem, st>>>(
        bd.Bd, bd.n, bd.b, shifts_dev, bd.stats, cnt_dev, (c128*)scratch);
  else
    k_band_ldlh_inertia<false><<<nshift, kInertiaThreads, smem, st>>>(
        bd.Bd, bd.n, bd.b, shifts_dev, bd.stats, cnt_dev, (c128*)scratch);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
