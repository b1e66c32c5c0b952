// Band ingest: LAPACK lower band (real or complex) -> diagonal-major complex128
// copy, plus ||B||_1 and the Gershgorin interval.
#include <algorithm>
#include <vector>

#include "fb_internal.h"

namespace fb {

// One thread per stored element in the caller's (column-major) order, so the
// reads are coalesced; writes go to row d of the diagonal-major copy.
__global__ void k_band_ingest(const double* __restrict__ ab, int64_t ldab, int cplx,
                              int64_t n, int b, int bsrc, c128* __restrict__ Bd) {
  int64_t total = (int64_t)(b + 1) * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = e / (b + 1);
    int d = (int)(e - j * (b + 1));
    c128 v = mk(0.0, 0.0);
    if (j + d < n && d <= bsrc) {
      if (cplx) {
        v = mk(ab[2 * (d + j * ldab)], ab[2 * (d + j * ldab) + 1]);
      } else {
        v = mk(ab[d + j * ldab], 0.0);
      }
      if (d == 0) v.y = 0.0;  // the diagonal of a Hermitian matrix is real
    }
    Bd[(int64_t)d * n + j] = v;
  }
}

// Column sums of |B| over the full Hermitian matrix: column j holds the
// lower entries B(j+d, j) and the upper ones conj(B(j, j-d)).
// Per block: max colsum, min(a_jj - R_j), max(a_jj + R_j), and the number of
// stored entries that are NaN or infinite.
__global__ void k_band_colstats(const c128* __restrict__ Bd, int64_t n, int b,
                                double* __restrict__ part) {
  __shared__ double s0[256], s1[256], s2[256], s3[256];
  double mx = 0.0, lo = 1e308, hi = -1e308, bad = 0.0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    double r = 0.0;
    for (int d = 1; d <= b; ++d) {
      if (j + d < n) {
        const c128 v = Bd[(int64_t)d * n + j];
        r += sqrt(cabs2(v));
        bad += (isfinite(v.x) && isfinite(v.y)) ? 0.0 : 1.0;
      }
      if (j - d >= 0) r += sqrt(cabs2(Bd[(int64_t)d * n + j - d]));
    }
    double a = Bd[j].x;
    bad += isfinite(a) ? 0.0 : 1.0;
    mx = fmax(mx, r + fabs(a));
    lo = fmin(lo, a - r);
    hi = fmax(hi, a + r);
  }
  int t = threadIdx.x;
  s0[t] = mx;
  s1[t] = lo;
  s2[t] = hi;
  s3[t] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      s0[t] = fmax(s0[t], s0[t + s]);
      s1[t] = fmin(s1[t], s1[t + s]);
      s2[t] = fmax(s2[t], s2[t + s]);
      s3[t] += s3[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[4 * blockIdx.x + 0] = s0[0];
    part[4 * blockIdx.x + 1] = s1[0];
    part[4 * blockIdx.x + 2] = s2[0];
    part[4 * blockIdx.x + 3] = s3[0];
  }
}

__global__ void k_band_colstats_final(const double* __restrict__ part, int nb,
                                      double* __restrict__ out) {
  __shared__ double s0[256], s1[256], s2[256], s3[256];
  int t = threadIdx.x;
  double mx = 0.0, lo = 1e308, hi = -1e308, bad = 0.0;
  for (int i = t; i < nb; i += blockDim.x) {
    mx = fmax(mx, part[4 * i]);
    lo = fmin(lo, part[4 * i + 1]);
    hi = fmax(hi, part[4 * i + 2]);
    bad += part[4 * i + 3];
  }
  s0[t] = mx;
  s1[t] = lo;
  s2[t] = hi;
  s3[t] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      s0[t] = fmax(s0[t], s0[t + s]);
      s1[t] = fmin(s1[t], s1[t + s]);
      s2[t] = fmax(s2[t], s2[t + s]);
      s3[t] += s3[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
    out[2] = s2[0];
    out[3] = s3[0];
  }
}

// Dense nb x nb blocks of the block-tridiagonal form of B (zero outside the
// band and beyond n).
__global__ void k_band_blocks(const c128* __restrict__ Bd, int64_t n, int b, int nb, int K,
                              c128* __restrict__ Bblk) {
  const int64_t total = (int64_t)K * 3 * nb * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t blk = e / ((int64_t)nb * nb);
    int rem = (int)(e - blk * nb * nb);
    int c = rem / nb, r = rem % nb;
    int k = (int)(blk / 3), sft = (int)(blk % 3) - 1;
    int64_t i = (int64_t)k * nb + r, j = (int64_t)(k + sft) * nb + c;
    c128 v = mk(0.0, 0.0);
    if (j >= 0 && i < n && j < n) {
      int64_t d = i - j;
      if (d >= 0 && d <= b) {
        v = Bd[d * n + j];
        if (d == 0) v.y = 0.0;
      } else if (d < 0 && -d <= b) {
        c128 u = Bd[(-d) * n + i];
        v = mk(u.x, -u.y);
      }
    }
    Bblk[e] = v;
  }
}

static const int kStatBlocks = 256;

int ingest_band(const fb_band* B, Band& out, Arena& ar, hipStream_t st, bool blocks) {
  // a diagonal matrix is handled as a band of width 1 with a zero sub-diagonal
  out.n = B->n;
  out.b = B->b > 0 ? B->b : 1;
  out.b0 = B->b;
  out.cplx = B->dtype == FB_COMPLEX128;
  out.Bd = ar.take<c128>((size_t)(out.b + 1) * B->n);
  out.stats = ar.take<double>(4);
  out.nb = (out.b + 15) / 16 * 16;
  out.K = (int)((out.n + out.nb - 1) / out.nb);
  out.Bblk = blocks ? ar.take<c128>((size_t)out.K * 3 * out.nb * out.nb) : nullptr;
  double* part = ar.take<double>(4 * kStatBlocks);
  if (ar.base == nullptr) return 0;
  if (!ar.fits()) return FB_ERR_NOMEM;
  int64_t total = (int64_t)(out.b + 1) * B->n;
  int grid = (int)((total + 255) / 256);
  if (grid > 65535 * 4) grid = 65535 * 4;
  k_band_ingest<<<grid, 256, 0, st>>>((const double*)B->ab, B->ldab, out.cplx ? 1 : 0,
                                      B->n, out.b, B->b, out.Bd);
  FB_HIP(hipGetLastError());
  k_band_colstats<<<kStatBlocks, 256, 0, st>>>(out.Bd, B->n, out.b, part);
  FB_HIP(hipGetLastError());
  k_band_colstats_final<<<1, 256, 0, st>>>(part, kStatBlocks, out.stats);
  FB_HIP(hipGetLastError());
  if (blocks) {
    int64_t tb = (int64_t)out.K * 3 * out.nb * out.nb;
    int g = (int)std::min<int64_t>((tb + 255) / 256, 65536);
    k_band_blocks<<<g, 256, 0, st>>>(out.Bd, out.n, out.b, out.nb, out.K, out.Bblk);
    FB_HIP(hipGetLastError());
  }
  double bad = 0.0;
  FB_HIP(hipMemcpyAsync(&bad, out.stats + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  if (bad != 0.0) return FB_ERR_NONFINITE;
  return 0;
}

// Number of NaN or infinite entries of a column-major block (real or
// complex), added to *count: workgroup (x, c) reads a stretch of column c,
// one contiguous run of rows x words doubles, so the scan runs at HBM rate.
__global__ void __launch_bounds__(256)
k_count_nonfinite(const double* __restrict__ p, int64_t rows, int64_t ld, int words,
                  int32_t* __restrict__ count) {
  const int64_t len = rows * words;
  const double* col = p + (int64_t)blockIdx.y * ld * words;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    bad += isfinite(col[e]) ? 0 : 1;
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

int check_finite_blocks(int nblk, const void* const* P, const int64_t* ld, const int32_t* cols,
                        int64_t rows, bool cplx, double* part_dev, hipStream_t st) {
  if (nblk <= 0) return 0;
  int32_t* cnt = reinterpret_cast<int32_t*>(part_dev);  // nblk counters
  FB_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nblk, st));
  const int words = cplx ? 2 : 1;
  const int64_t len = rows * words;
  const int gx = (int)std::min<int64_t>((len + 1023) / 1024, 64);  // about 4 doubles per thread
  for (int i = 0; i < nblk; ++i) {
    if (cols[i] <= 0) continue;
    for (int c0 = 0; c0 < cols[i]; c0 += 65535) {
      const int nc = std::min(cols[i] - c0, 65535);
      k_count_nonfinite<<<dim3(gx, nc), 256, 0, st>>>(
          (const double*)P[i] + (int64_t)c0 * ld[i] * words, rows, ld[i], words, cnt + i);
      FB_HIP(hipGetLastError());
    }
  }
  std::vector<int32_t> h(nblk);
  FB_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * nblk, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  for (int32_t v : h)
    if (v != 0) return FB_ERR_NONFINITE;
  return 0;
}

int band_stats_host(const Band& bd, double* out3, hipStream_t st) {
  FB_HIP(hipMemcpyAsync(out3, bd.stats, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  return 0;
}

}  // namespace fb
