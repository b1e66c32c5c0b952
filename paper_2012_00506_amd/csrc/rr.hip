// Rayleigh-Ritz support kernels (FP64): band products, eigen-residuals,
// column gathers, and a cyclic Jacobi eigensolver for the reduced Hermitian
// problems A_q W = W Lambda (Section 2.2, "The FEAST Algorithm").
#include "rr.h"
#include "prof.h"

namespace fb {

// ---------------------------------------------------------------- fills / copies
__global__ void k_fill_c128(c128* __restrict__ p, int64_t rows, int64_t cols, int64_t ld) {
  int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t c = e / rows, r = e - c * rows;
    p[c * ld + r] = mk(0.0, 0.0);
  }
}

int fill_zero(c128* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  int64_t total = rows * cols;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  k_fill_c128<<<grid, 256, 0, st>>>(p, rows, cols, ld);
  FB_HIP(hipGetLastError());
  return 0;
}

// dst[:, k] = src[:, idx[k]] * (scale ? scale[k] : 1); real_src: src is double
__global__ void __launch_bounds__(256)
k_accumulate_pairs(const AccJob* __restrict__ jobs, int64_t n) {
  const AccJob& J = jobs[blockIdx.y];
  const int64_t total = n * J.m;
  const int np = J.np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n, row = e - col * n;
    c128* q = J.Q + col * J.ldq + row;
    c128 acc = J.init ? mk(0.0, 0.0) : gld(q);
    for (int p = 0; p < np; ++p) {
      c128 wv = J.w[p] * gld(J.X[p] + col * J.ldx + row);
      if (J.acc_real)
        acc.x += 2.0 * wv.x;
      else
        acc = acc + wv;
    }
    gst(q, acc);
  }
}

int accumulate_pairs(const AccJob* jobs_dev, int njobs, int64_t n, int max_m, hipStream_t st) {
  if (njobs <= 0 || max_m <= 0) return 0;
  int64_t blocks = std::min<int64_t>((n * max_m + 255) / 256, 2048);
  k_accumulate_pairs<<<dim3((unsigned)blocks, njobs), 256, 0, st>>>(jobs_dev, n);
  FB_HIP(hipGetLastError());
  return 0;
}

__global__ void k_gather_cols(const void* __restrict__ src, int64_t lds, int real_src,
                              c128* __restrict__ dst, int64_t ldd, int64_t rows, int cols,
                              const int32_t* __restrict__ idx, const double* __restrict__ scale) {
  int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(e / rows);
    int64_t r = e - (int64_t)k * rows;
    int64_t sc = idx ? idx[k] : k;
    c128 v = real_src ? mk(((const double*)src)[sc * lds + r], 0.0)
                      : ((const c128*)src)[sc * lds + r];
    if (scale) v = scale[k] * v;
    dst[(int64_t)k * ldd + r] = v;
  }
}

int gather_cols(const void* src, int64_t lds, bool real_src, c128* dst, int64_t ldd,
                int64_t rows, int cols, const int32_t* idx_dev, const double* scale_dev,
                hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  int64_t total = rows * cols;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  k_gather_cols<<<grid, 256, 0, st>>>(src, lds, real_src ? 1 : 0, dst, ldd, rows, cols, idx_dev,
                                      scale_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

// complex128 columns -> caller's block (complex, or the real part)
__global__ void k_store_cols(const c128* __restrict__ src, int64_t lds, void* __restrict__ dst,
                             int64_t ldd, int real_dst, int64_t rows, int cols,
                             const int32_t* __restrict__ idx) {
  int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(e / rows);
    int64_t r = e - (int64_t)k * rows;
    c128 v = src[(int64_t)(idx ? idx[k] : k) * lds + r];
    if (real_dst)
      ((double*)dst)[(int64_t)k * ldd + r] = v.x;
    else
      ((c128*)dst)[(int64_t)k * ldd + r] = v;
  }
}

int store_cols(const c128* src, int64_t lds, void* dst, int64_t ldd, bool real_dst, int64_t rows,
               int cols, const int32_t* idx_dev, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  int64_t total = rows * cols;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  k_store_cols<<<grid, 256, 0, st>>>(src, lds, dst, ldd, real_dst ? 1 : 0, rows, cols, idx_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

// A <- (A + A^H) / 2 for an m x m matrix
__global__ void k_hermitize(c128* __restrict__ A, int m, int64_t lda) {
  int64_t total = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    if (i > j) continue;
    c128 a = A[(int64_t)j * lda + i], b = A[(int64_t)i * lda + j];
    c128 h = mk(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    A[(int64_t)j * lda + i] = h;
    A[(int64_t)i * lda + j] = mk(h.x, i == j ? 0.0 : -h.y);
    if (i == j) A[(int64_t)j * lda + i] = mk(h.x, 0.0);
  }
}

int hermitize(c128* A, int m, int64_t lda, hipStream_t st) {
  if (m <= 0) return 0;
  int64_t total = (int64_t)m * m;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  k_hermitize<<<grid, 256, 0, st>>>(A, m, lda);
  FB_HIP(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------- band products
// Y = B X (or Y = B X - X diag(lam) with per-column norms when lam != NULL).
static const int kBmRows = 256;

__global__ void __launch_bounds__(256)
k_band_matmul(const c128* __restrict__ Bd, int64_t n, int b, const c128* __restrict__ X,
              int64_t ldx, c128* __restrict__ Y, int64_t ldy, int m) {
  const int64_t i = blockIdx.x * (int64_t)kBmRows + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= m) return;
  const c128* x = X + (int64_t)c * ldx;
  c128 acc = mk(Bd[i].x * x[i].x, Bd[i].x * x[i].y);
  for (int d = 1; d <= b; ++d) {
    if (i - d >= 0) cmac(acc, Bd[(int64_t)d * n + i - d], x[i - d]);
    if (i + d < n) cmacc(acc, Bd[(int64_t)d * n + i], x[i + d]);
  }
  Y[(int64_t)c * ldy + i] = acc;
}

int band_matmul(const Band& bd, const c128* X, int64_t ldx, c128* Y, int64_t ldy, int m,
                hipStream_t st) {
  if (m <= 0) return 0;
  ProfScope ps(FB_PROF_BANDMM, st, 8.0 * (2.0 * bd.b + 1.0) * bd.n * m);
  for (int c0 = 0; c0 < m; c0 += 65535) {
    int mc = std::min(65535, m - c0);
    dim3 grid((unsigned)((bd.n + kBmRows - 1) / kBmRows), (unsigned)mc);
    k_band_matmul<<<grid, kBmRows, 0, st>>>(bd.Bd, bd.n, bd.b, X + (int64_t)c0 * ldx, ldx,
                                            Y + (int64_t)c0 * ldy, ldy, mc);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

// per column: sum |B x - lam x|^2 and sum |x|^2 over a row chunk
static const int kErChunk = 4096;

__global__ void __launch_bounds__(256)
k_eig_resid_part(const c128* __restrict__ Bd, int64_t n, int b, const c128* __restrict__ X,
                 int64_t ldx, const double* __restrict__ lam, double* __restrict__ part, int m,
                 int nchunk) {
  const int c = blockIdx.y, ch = blockIdx.x;
  const int t = threadIdx.x;
  __shared__ double red[2][256];
  double rr = 0.0, xx = 0.0;
  if (c < m) {
    const c128* x = X + (int64_t)c * ldx;
    const double l = lam[c];
    int64_t i0 = (int64_t)ch * kErChunk, i1 = std::min<int64_t>(i0 + kErChunk, n);
    for (int64_t i = i0 + t; i < i1; i += 256) {
      c128 xi = x[i];
      c128 acc = mk((Bd[i].x - l) * xi.x, (Bd[i].x - l) * xi.y);
      for (int d = 1; d <= b; ++d) {
        if (i - d >= 0) cmac(acc, Bd[(int64_t)d * n + i - d], x[i - d]);
        if (i + d < n) cmacc(acc, Bd[(int64_t)d * n + i], x[i + d]);
      }
      rr += cabs2(acc);
      xx += cabs2(xi);
    }
  }
  red[0][t] = rr;
  red[1][t] = xx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
    }
    __syncthreads();
  }
  if (t == 0 && c < m) {
    part[((size_t)c * nchunk + ch) * 2] = red[0][0];
    part[((size_t)c * nchunk + ch) * 2 + 1] = red[1][0];
  }
}

__global__ void k_eig_resid_final(const double* __restrict__ part, int m, int nchunk,
                                  const double* __restrict__ stats, double* __restrict__ res) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double rr = 0.0, xx = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    rr += part[((size_t)c * nchunk + ch) * 2];
    xx += part[((size_t)c * nchunk + ch) * 2 + 1];
  }
  double nrm = stats[0] > 0.0 ? stats[0] : 1.0;
  res[c] = xx > 0.0 ? sqrt(rr / xx) / nrm : 1e300;
}

size_t eig_resid_part_doubles(int64_t n, int m) {
  int nchunk = (int)((n + kErChunk - 1) / kErChunk);
  return (size_t)m * nchunk * 2;
}

int eig_residuals(const Band& bd, const c128* X, int64_t ldx, const double* lam, int m,
                  double* part, double* res, hipStream_t st) {
  if (m <= 0) return 0;
  int nchunk = (int)((bd.n + kErChunk - 1) / kErChunk);
  for (int c0 = 0; c0 < m; c0 += 65535) {
    int mc = std::min(65535, m - c0);
    dim3 grid((unsigned)nchunk, (unsigned)mc);
    k_eig_resid_part<<<grid, 256, 0, st>>>(bd.Bd, bd.n, bd.b, X + (int64_t)c0 * ldx, ldx,
                                           lam + c0, part + (size_t)c0 * nchunk * 2, mc, nchunk);
    FB_HIP(hipGetLastError());
  }
  k_eig_resid_final<<<(m + 255) / 256, 256, 0, st>>>(part, m, nchunk, bd.stats, res);
  FB_HIP(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------- Jacobi
// Two-sided cyclic Jacobi for Hermitian A (m x m, column-major, in place),
// one workgroup per matrix.  Each round applies the rotations of m/2 disjoint
// pairs (circle-method ordering): rotation parameters from the current A,
// then A <- J^H A J one 2x2 block at a time (every block of the pair-of-pairs
// grid is independent) and V <- V J.  The rotation of a pair (p, q) first
// makes A(p,q) real with the phase e^{-i arg A(p,q)} on q, then applies the
// symmetric Schur rotation t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = (A(q,q) - A(p,p)) / (2 |A(p,q)|).  Sweeps stop when
// ||offdiag(A)||_F <= tol ||A||_F.  On exit w holds the eigenvalues in
// ascending order and W the matching eigenvectors (columns of V sorted).
static const int kJacThreads = 1024;
static const int kJacMaxPairs = 2048;

__device__ __forceinline__ int rr_player(int pos, int r, int mp) {
  // circle method: position 0 fixed, the others rotate by r
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (mp - 1);
}

__global__ void __launch_bounds__(kJacThreads)
k_jacobi(JacobiJob* __restrict__ jobs, int max_sweeps, double tol) {
  __shared__ double s_cs[kJacMaxPairs];
  __shared__ double s_sn[kJacMaxPairs];
  __shared__ c128 s_e[kJacMaxPairs];
  __shared__ int s_p[kJacMaxPairs + 1];
  __shared__ int s_q[kJacMaxPairs + 1];
  __shared__ double red[kJacThreads];
  __shared__ double s_fro2, s_off2;
  JacobiJob jb = jobs[blockIdx.x];
  const int m = jb.m;
  const int t = threadIdx.x;
  c128* A = jb.A;
  c128* V = jb.V;
  const int64_t lda = jb.lda, ldv = jb.ldv;
  if (m <= 0) return;
  const int mp = m + (m & 1);     // even number of players (m = dummy if odd)
  const int np = mp / 2;

  for (int64_t e = t; e < (int64_t)m * m; e += blockDim.x) {
    int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    V[(int64_t)j * ldv + i] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  int sweeps = 0;
  for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
    // convergence test
    double f = 0.0, o = 0.0;
    for (int64_t e = t; e < (int64_t)m * m; e += blockDim.x) {
      int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
      double a = cabs2(A[(int64_t)j * lda + i]);
      f += a;
      if (i != j) o += a;
    }
    red[t] = f;
    __syncthreads();
    for (int s = kJacThreads / 2; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) s_fro2 = red[0];
    __syncthreads();
    red[t] = o;
    __syncthreads();
    for (int s = kJacThreads / 2; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) s_off2 = red[0];
    __syncthreads();
    if (s_off2 <= tol * tol * s_fro2 || sweep == max_sweeps || m == 1) break;
    ++sweeps;
    for (int r = 0; r < mp - 1; ++r) {
      // pairs of this round and their rotations
      for (int k = t; k < np; k += blockDim.x) {
        int a = rr_player(k, r, mp), bq = rr_player(mp - 1 - k, r, mp);
        int p = a < bq ? a : bq, q = a < bq ? bq : a;
        s_p[k] = p;
        s_q[k] = q;
        double cs = 1.0, sn = 0.0;
        c128 e = mk(1.0, 0.0);
        if (q < m) {
          c128 c = A[(int64_t)q * lda + p];
          double ac = sqrt(cabs2(c));
          if (ac > 1e-300) {
            double app = A[(int64_t)p * lda + p].x, aqq = A[(int64_t)q * lda + q].x;
            double tau = (aqq - app) / (2.0 * ac);
            double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            cs = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * cs;
            e = mk(c.x / ac, -c.y / ac);  // e^{-i arg c}
          }
        }
        s_cs[k] = cs;
        s_sn[k] = sn;
        s_e[k] = e;
      }
      __syncthreads();
      // A <- J^H A J by 2x2 blocks (pair k rows, pair l columns)
      for (int64_t e2 = t; e2 < (int64_t)np * np; e2 += blockDim.x) {
        int l = (int)(e2 / np), k = (int)(e2 - (int64_t)l * np);
        int pk = s_p[k], qk = s_q[k], pl = s_p[l], ql = s_q[l];
        bool qkv = qk < m, qlv = ql < m;
        c128 a00 = A[(int64_t)pl * lda + pk];
        c128 a10 = qkv ? A[(int64_t)pl * lda + qk] : mk(0.0, 0.0);
        c128 a01 = qlv ? A[(int64_t)ql * lda + pk] : mk(0.0, 0.0);
        c128 a11 = (qkv && qlv) ? A[(int64_t)ql * lda + qk] : mk(0.0, 0.0);
        // right: columns (pl, ql) times [[cs, sn], [-sn e, cs e]]
        double cl = s_cs[l], sl = s_sn[l];
        c128 el = s_e[l];
        c128 b00 = cl * a00 - sl * (el * a01), b01 = sl * a00 + cl * (el * a01);
        c128 b10 = cl * a10 - sl * (el * a11), b11 = sl * a10 + cl * (el * a11);
        // left: rows (pk, qk) times [[cs, -sn conj(e)], [sn, cs conj(e)]]
        double ck = s_cs[k], sk = s_sn[k];
        c128 ek = cconj(s_e[k]);
        c128 c00 = ck * b00 - sk * (ek * b10), c10 = sk * b00 + ck * (ek * b10);
        c128 c01 = ck * b01 - sk * (ek * b11), c11 = sk * b01 + ck * (ek * b11);
        A[(int64_t)pl * lda + pk] = c00;
        if (qkv) A[(int64_t)pl * lda + qk] = c10;
        if (qlv) A[(int64_t)ql * lda + pk] = c01;
        if (qkv && qlv) A[(int64_t)ql * lda + qk] = c11;
      }
      // V <- V J (columns p, q of every row)
      for (int64_t e2 = t; e2 < (int64_t)np * m; e2 += blockDim.x) {
        int k = (int)(e2 / m), i = (int)(e2 - (int64_t)k * m);
        int p = s_p[k], q = s_q[k];
        if (q >= m) continue;
        double cs = s_cs[k], sn = s_sn[k];
        c128 e = s_e[k];
        c128 vp = V[(int64_t)p * ldv + i], vq = V[(int64_t)q * ldv + i];
        V[(int64_t)p * ldv + i] = cs * vp - sn * (e * vq);
        V[(int64_t)q * ldv + i] = sn * vp + cs * (e * vq);
      }
      __syncthreads();
    }
  }
  // eigenvalues ascending (rank by value, ties by index), vectors follow
  for (int i = t; i < m; i += blockDim.x) {
    double wi = A[(int64_t)i * lda + i].x;
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      double wj = A[(int64_t)j * lda + j].x;
      rank += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
    }
    jb.w[rank] = wi;
    jb.order[rank] = i;
  }
  if (t == 0 && jb.sweeps) *jb.sweeps = sweeps;
  __syncthreads();
  for (int64_t e = t; e < (int64_t)m * m; e += blockDim.x) {
    int k = (int)(e / m), i = (int)(e - (int64_t)k * m);
    jb.W[(int64_t)k * jb.ldw + i] = V[(int64_t)jb.order[k] * ldv + i];
  }
}

int launch_jacobi(int njobs, JacobiJob* jobs_dev, int max_sweeps, double tol, hipStream_t st) {
  if (njobs <= 0) return 0;
  ProfScope ps(FB_PROF_JACOBI, st, 0.0);
  k_jacobi<<<njobs, kJacThreads, 0, st>>>(jobs_dev, max_sweeps, tol);
  FB_HIP(hipGetLastError());
  return 0;
}

// s -> s^{-1/2} for the kept directions (descending order of kept columns is
// irrelevant; idx lists them), keep = s > drop * max(s)
__global__ void k_gram_keep(const double* __restrict__ s, int m, double drop,
                            int32_t* __restrict__ idx, double* __restrict__ scale,
                            int32_t* __restrict__ kept) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = 0.0;
  for (int i = 0; i < m; ++i) mx = fmax(mx, s[i]);
  int k = 0;
  // eigenvalues come ascending: keep the large ones, largest last
  for (int i = 0; i < m; ++i)
    if (s[i] > drop * mx && mx > 0.0) {
      idx[k] = i;
      scale[k] = 1.0 / sqrt(s[i]);
      ++k;
    }
  *kept = k;
}

// 2-norm of every column of the n x m block X: one workgroup per column
__global__ void __launch_bounds__(256)
k_col_norms(const c128* __restrict__ X, int64_t n, int64_t ldx, double* __restrict__ nrm) {
  __shared__ double red[4];
  const c128* x = X + (int64_t)blockIdx.x * ldx;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) ss += cabs2(x[i]);
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// keep = nrm > thr * max(nrm): idx lists the kept columns in order, scale = 1 / nrm
__global__ void k_norm_keep(const double* __restrict__ nrm, int m, double thr,
                            int32_t* __restrict__ idx, double* __restrict__ scale,
                            int32_t* __restrict__ kept) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = 0.0;
  for (int i = 0; i < m; ++i) mx = fmax(mx, nrm[i]);
  int k = 0;
  for (int i = 0; i < m; ++i)
    if (nrm[i] > thr * mx && mx > 0.0) {
      idx[k] = i;
      scale[k] = 1.0 / nrm[i];
      ++k;
    }
  *kept = k;
}

int col_norm_keep(const c128* X, int64_t n, int64_t ldx, int m, double thr, double* nrm,
                  int32_t* idx, double* scale, int32_t* kept, hipStream_t st) {
  if (m <= 0) return 0;
  k_col_norms<<<m, 256, 0, st>>>(X, n, ldx, nrm);
  FB_HIP(hipGetLastError());
  k_norm_keep<<<1, 64, 0, st>>>(nrm, m, thr, idx, scale, kept);
  FB_HIP(hipGetLastError());
  return 0;
}

int gram_keep(const double* s, int m, double drop, int32_t* idx, double* scale, int32_t* kept,
              hipStream_t st) {
  k_gram_keep<<<1, 64, 0, st>>>(s, m, drop, idx, scale, kept);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
