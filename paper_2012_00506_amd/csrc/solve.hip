// Multi-right-hand-side solves with the block form of the band LU factors.
//
// N: x = A^{-1} y.  Forward, block k on the window rows kb .. kb+2b-1:
//      z = P y_win; y_top = Lh11^{-1} z_top; carry = z_bot - Lh21 y_top
//    Backward: x_k = U(k,k)^{-1} (y_k - U(k,k+1) x_{k+1} - U(k,k+2) x_{k+2}).
// H: x = A^{-H} y.  Forward with U^H:
//      w_k = U(k,k)^{-H} (y_k - U(k-1,k)^H w_{k-1} - U(k-2,k)^H w_{k-2})
//    Backward, k descending on the window [w_k ; carry]:
//      top = Lh11^{-H} (w_k - Lh21^H carry); x_win = P^T [top ; carry]
//    (rows kb+b .. kb+2b-1 of x_win are final, rows kb .. kb+b-1 carry on).
// One workgroup per job (system, direction, tile of T columns); the tile's
// window and carries live in LDS.  Inputs and outputs are complex128; the
// arithmetic is in R (float: complex64 path, double: complex128 path).
#include "fb_internal.h"
#include "solve_job.h"
#include "prof.h"

namespace fb {

static const int kSolveThreads = 256;

template <typename R>
__device__ __forceinline__ cx<R> ld_in(const c128* p) {
  c128 v = *p;
  return mk<R>((R)v.x, (R)v.y);
}

template <typename R, int T>
__global__ void __launch_bounds__(kSolveThreads)
k_band_solve(const cx<R>* __restrict__ mats, const int16_t* __restrict__ permg, int64_t n,
             int b, int K, const SolveJob* __restrict__ jobs) {
  extern __shared__ char lds_raw[];
  cx<R>* S = reinterpret_cast<cx<R>*>(lds_raw);
  const SolveJob jb = jobs[blockIdx.x];
  const int t = threadIdx.x;
  const int c = t % T;               // tile column of this thread
  const int r0 = t / T;              // first row; rows r0 + RS*i
  const int RS = kSolveThreads / T;
  const int nrow = (b + RS - 1) / RS;
  const bool colok = c < jb.ncol;
  const size_t bb = (size_t)b * b;
  const cx<R>* F = mats + (size_t)jb.sys * K * 5 * bb;
  const int16_t* P = permg + (size_t)jb.sys * K * 2 * b;
  const c128* in = jb.in + (int64_t)jb.col0 * jb.ldin;
  c128* mid = jb.mid + (int64_t)jb.col0 * jb.ldmid;
  c128* out = jb.out + (int64_t)jb.col0 * jb.ldout;
  const int64_t npad = (int64_t)K * b;
  constexpr int MAXR = 16;  // rows per thread: b <= 16 * RS

  c128* accp = jb.acc ? jb.acc + (int64_t)jb.col0 * jb.ldacc : nullptr;
  // final value of a solution entry: store (or add) it, and fold it into the
  // node sum when accumulating
  auto emit = [&](int64_t row, c128 v) {
    c128* o = out + (int64_t)c * jb.ldout + row;
    *o = jb.add ? *o + v : v;
    if (accp) {
      c128* a = accp + (int64_t)c * jb.ldacc + row;
      c128 wv = jb.w * v;
      if (jb.acc_real) wv = mk(2.0 * wv.x, 0.0);
      *a = *a + wv;
    }
  };

  auto load_in = [&](int64_t row) -> cx<R> {
    if (!colok || row >= n) return mk<R>(0, 0);
    return ld_in<R>(in + (int64_t)c * jb.ldin + row);
  };

  if (jb.dir == 0) {
    // ------------------------------------------------------------ N forward
    cx<R>* Win = S;                  // 2b x T
    cx<R>* Yt = S + 2 * b * T;       // b x T
    for (int r = r0; r < 2 * b; r += RS) Win[r * T + c] = load_in(r);
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      const cx<R>* Li = F + ((size_t)k * 5 + 0) * bb;
      const cx<R>* L21 = F + ((size_t)k * 5 + 1) * bb;
      const int16_t* pk = P + (size_t)k * 2 * b;
      // y_top = Li * (P win)_top
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        cx<R> acc = mk<R>(0, 0);
        for (int q = 0; q <= r; ++q) cmac(acc, Li[(size_t)q * b + r], Win[pk[q] * T + c]);
        Yt[r * T + c] = acc;
      }
      __syncthreads();
      // carry = (P win)_bot - L21 * y_top
      cx<R> nb[MAXR];
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        cx<R> acc = Win[pk[b + r] * T + c];
        for (int q = 0; q < b; ++q) {
          cx<R> l = L21[(size_t)q * b + r];
          cx<R> y = Yt[q * T + c];
          acc.x -= l.x * y.x - l.y * y.y;
          acc.y -= l.x * y.y + l.y * y.x;
        }
        nb[i] = acc;
        int64_t row = (int64_t)k * b + r;
        if (colok && row < n) mid[(int64_t)c * jb.ldmid + row] = mk((double)Yt[r * T + c].x,
                                                                    (double)Yt[r * T + c].y);
      }
      __syncthreads();
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        Win[r * T + c] = nb[i];
        Win[(b + r) * T + c] = load_in((int64_t)(k + 2) * b + r);
      }
      __syncthreads();
    }
    // ------------------------------------------------------------ N backward
    cx<R>* X1 = S;            // x_{k+1}
    cx<R>* X2 = S + b * T;    // x_{k+2}
    cx<R>* V = S + 2 * b * T;
    for (int r = r0; r < b; r += RS) {
      X1[r * T + c] = mk<R>(0, 0);
      X2[r * T + c] = mk<R>(0, 0);
    }
    __syncthreads();
    for (int k = K - 1; k >= 0; --k) {
      const cx<R>* Ui = F + ((size_t)k * 5 + 2) * bb;
      const cx<R>* U1 = F + ((size_t)k * 5 + 3) * bb;
      const cx<R>* U2 = F + ((size_t)k * 5 + 4) * bb;
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        int64_t row = (int64_t)k * b + r;
        cx<R> acc = (colok && row < n) ? ld_in<R>(mid + (int64_t)c * jb.ldmid + row) : mk<R>(0, 0);
        if (k + 1 < K)
          for (int q = 0; q < b; ++q) {
            cx<R> u = U1[(size_t)q * b + r];
            cx<R> x = X1[q * T + c];
            acc.x -= u.x * x.x - u.y * x.y;
            acc.y -= u.x * x.y + u.y * x.x;
          }
        if (k + 2 < K)
          for (int q = 0; q <= r; ++q) {
            cx<R> u = U2[(size_t)q * b + r];
            cx<R> x = X2[q * T + c];
            acc.x -= u.x * x.x - u.y * x.y;
            acc.y -= u.x * x.y + u.y * x.x;
          }
        V[r * T + c] = acc;
      }
      __syncthreads();
      cx<R> xr[MAXR];
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        cx<R> acc = mk<R>(0, 0);
        for (int q = r; q < b; ++q) cmac(acc, Ui[(size_t)q * b + r], V[q * T + c]);
        xr[i] = acc;
        int64_t row = (int64_t)k * b + r;
        if (colok && row < n) emit(row, mk((double)acc.x, (double)acc.y));
      }
      __syncthreads();
      // rotate carries: x_{k+2} <- x_{k+1}, x_{k+1} <- x_k
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        X2[r * T + c] = X1[r * T + c];
      }
      __syncthreads();
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        X1[r * T + c] = xr[i];
      }
      __syncthreads();
    }
  } else {
    // ------------------------------------------------------------ H forward (U^H)
    cx<R>* W1 = S;            // w_{k-1}
    cx<R>* W2 = S + b * T;    // w_{k-2}
    cx<R>* V = S + 2 * b * T;
    for (int r = r0; r < b; r += RS) {
      W1[r * T + c] = mk<R>(0, 0);
      W2[r * T + c] = mk<R>(0, 0);
    }
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      const cx<R>* Ui = F + ((size_t)k * 5 + 2) * bb;
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        int64_t row = (int64_t)k * b + r;
        cx<R> acc = load_in(row);
        if (k >= 1) {
          const cx<R>* U1 = F + ((size_t)(k - 1) * 5 + 3) * bb;  // U(k-1,k)
          // (U1^H)[r][q] = conj(U1[q][r]) = conj(U1_colmajor[r*b + q])
          for (int q = 0; q < b; ++q) {
            cx<R> u = U1[(size_t)r * b + q];
            cx<R> w = W1[q * T + c];
            acc.x -= u.x * w.x + u.y * w.y;
            acc.y -= u.x * w.y - u.y * w.x;
          }
        }
        if (k >= 2) {
          const cx<R>* U2 = F + ((size_t)(k - 2) * 5 + 4) * bb;  // U(k-2,k), lower
          for (int q = r; q < b; ++q) {
            cx<R> u = U2[(size_t)r * b + q];
            cx<R> w = W2[q * T + c];
            acc.x -= u.x * w.x + u.y * w.y;
            acc.y -= u.x * w.y - u.y * w.x;
          }
        }
        V[r * T + c] = acc;
      }
      __syncthreads();
      cx<R> wr[MAXR];
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        // (Ui^H)[r][q] = conj(Ui[q][r]), Ui upper so q <= r
        cx<R> acc = mk<R>(0, 0);
        for (int q = 0; q <= r; ++q) cmacc(acc, Ui[(size_t)r * b + q], V[q * T + c]);
        wr[i] = acc;
        int64_t row = (int64_t)k * b + r;
        if (colok && row < n) mid[(int64_t)c * jb.ldmid + row] = mk((double)acc.x, (double)acc.y);
      }
      __syncthreads();
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        W2[r * T + c] = W1[r * T + c];
      }
      __syncthreads();
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        W1[r * T + c] = wr[i];
      }
      __syncthreads();
    }
    // ------------------------------------------------------------ H backward (L^H)
    cx<R>* V2 = S;                 // 2b x T: [top ; carry]
    cx<R>* C = S + 2 * b * T;      // carry (next)
    cx<R>* T1 = S + 3 * b * T;
    for (int r = r0; r < b; r += RS) V2[(b + r) * T + c] = mk<R>(0, 0);
    __syncthreads();
    for (int k = K - 1; k >= 0; --k) {
      const cx<R>* Li = F + ((size_t)k * 5 + 0) * bb;
      const cx<R>* L21 = F + ((size_t)k * 5 + 1) * bb;
      const int16_t* pk = P + (size_t)k * 2 * b;
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        int64_t row = (int64_t)k * b + r;
        cx<R> acc = (colok && row < n) ? ld_in<R>(mid + (int64_t)c * jb.ldmid + row) : mk<R>(0, 0);
        // (L21^H)[r][q] = conj(L21[q][r]) = conj(L21_colmajor[r*b + q])
        for (int q = 0; q < b; ++q) {
          cx<R> l = L21[(size_t)r * b + q];
          cx<R> v = V2[(b + q) * T + c];
          acc.x -= l.x * v.x + l.y * v.y;
          acc.y -= l.x * v.y - l.y * v.x;
        }
        T1[r * T + c] = acc;
      }
      __syncthreads();
      cx<R> tr[MAXR];
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        // (Li^H)[r][q] = conj(Li[q][r]), Li unit lower so q >= r
        cx<R> acc = mk<R>(0, 0);
        for (int q = r; q < b; ++q) cmacc(acc, Li[(size_t)r * b + q], T1[q * T + c]);
        tr[i] = acc;
      }
      __syncthreads();
      for (int i = 0; i < nrow; ++i) {
        int r = r0 + RS * i;
        if (r >= b) break;
        V2[r * T + c] = tr[i];
      }
      __syncthreads();
      // x_win = P^T [top ; carry]: row perm[i] of the window gets V2[i]
      for (int i = r0; i < 2 * b; i += RS) {
        int d = pk[i];
        cx<R> v = V2[i * T + c];
        if (d >= b) {
          int64_t row = (int64_t)k * b + d;
          if (colok && row < n) emit(row, mk((double)v.x, (double)v.y));
        } else {
          C[d * T + c] = v;
        }
      }
      __syncthreads();
      for (int r = r0; r < b; r += RS) V2[(b + r) * T + c] = C[r * T + c];
      __syncthreads();
    }
    // rows 0 .. b-1 are final
    for (int r = r0; r < b; r += RS) {
      if (colok && r < n) {
        cx<R> v = V2[(b + r) * T + c];
        emit(r, mk((double)v.x, (double)v.y));
      }
    }
  }
  (void)npad;
}

template <typename R>
int solve_tile(int b) {
  // LDS holds 4 b x T blocks (window, carries, temporaries)
  return (size_t)4 * b * 32 * sizeof(cx<R>) <= 160 * 1024 ? 32 : 16;
}

template <typename R, int T>
static int launch_solve_t(const cx<R>* mats, const int16_t* perm, int64_t n, int b, int njobs,
                          const SolveJob* jobs_dev, double work, hipStream_t st) {
  ProfScope ps(FB_PROF_SOLVE, st, work);
  const int K = (int)((n + b - 1) / b);
  if (b > 16 * (kSolveThreads / T)) return FB_ERR_INTERNAL;
  size_t smem = (size_t)4 * b * T * sizeof(cx<R>);
  (void)hipFuncSetAttribute((const void*)k_band_solve<R, T>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
  for (int j0 = 0; j0 < njobs; j0 += 1 << 20) {
    int nj = njobs - j0 < (1 << 20) ? njobs - j0 : (1 << 20);
    k_band_solve<R, T><<<nj, kSolveThreads, smem, st>>>(mats, perm, n, b, K, jobs_dev + j0);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

template <typename R>
int launch_solve_jobs(const cx<R>* mats, const int16_t* perm, int64_t n, int b, int njobs,
                      const SolveJob* jobs_dev, double work, hipStream_t st) {
  if (njobs <= 0) return 0;
  if (solve_tile<R>(b) == 32)
    return launch_solve_t<R, 32>(mats, perm, n, b, njobs, jobs_dev, work, st);
  return launch_solve_t<R, 16>(mats, perm, n, b, njobs, jobs_dev, work, st);
}

template int solve_tile<float>(int);
template int solve_tile<double>(int);

template int launch_solve_jobs<float>(const c64*, const int16_t*, int64_t, int, int,
                                      const SolveJob*, double, hipStream_t);
template int launch_solve_jobs<double>(const c128*, const int16_t*, int64_t, int, int,
                                       const SolveJob*, double, hipStream_t);

// ---------------------------------------------------------------- residual
// r = y - (zz x - B x) in FP64 with zz = z (N) or conj(z) (H), for the
// columns of a job; per (job, row chunk, column): sum |r|^2 and sum |y|^2.
static const int kResRows = 64;
static const int kResChunk = 2048;

__global__ void __launch_bounds__(256)
k_shift_residual(const c128* __restrict__ Bd, int64_t n, int b, const ResJob* __restrict__ jobs,
                 double* __restrict__ part, int nchunk) {
  const ResJob jb = jobs[blockIdx.y];
  const int chunk = blockIdx.x;
  const int t = threadIdx.x;
  const int lr = t % kResRows;       // row lane
  const int lc = t / kResRows;       // column lane (4)
  __shared__ double red[2][256];
  for (int cc = 0; cc < 32; cc += 4) {
    int c = cc + lc;
    double rr = 0.0, yy = 0.0;
    if (c < jb.ncol) {
      const c128* x = jb.x + (int64_t)(jb.col0 + c) * jb.ldx;
      const c128* y = jb.y + (int64_t)(jb.col0 + c) * jb.ldy;
      c128* r = jb.r + (int64_t)(jb.col0 + c) * jb.ldr;
      int64_t i0 = (int64_t)chunk * kResChunk;
      int64_t i1 = i0 + kResChunk < n ? i0 + kResChunk : n;
      for (int64_t i = i0 + lr; i < i1; i += kResRows) {
        c128 xi = x[i];
        // (B x)_i
        c128 acc = mk(Bd[i].x * xi.x, Bd[i].x * xi.y);
        for (int d = 1; d <= b; ++d) {
          if (i - d >= 0) cmac(acc, Bd[(int64_t)d * n + i - d], x[i - d]);
          if (i + d < n) cmacc(acc, Bd[(int64_t)d * n + i], x[i + d]);
        }
        c128 zz = jb.dir ? mk(jb.z.x, -jb.z.y) : jb.z;
        c128 yi = y[i];
        c128 ri = yi - (zz * xi - acc);
        r[i] = ri;
        rr += cabs2(ri);
        yy += cabs2(yi);
      }
    }
    red[0][t] = rr;
    red[1][t] = yy;
    __syncthreads();
    for (int s = kResRows / 2; s > 0; s >>= 1) {
      if (lr < s) {
        red[0][t] += red[0][t + s];
        red[1][t] += red[1][t + s];
      }
      __syncthreads();
    }
    if (lr == 0 && c < 32) {
      size_t o = (((size_t)blockIdx.y * nchunk + chunk) * 32 + c) * 2;
      part[o] = red[0][t];
      part[o + 1] = red[1][t];
    }
    __syncthreads();
  }
}

// per job: max over its columns of sqrt(sum|r|^2 / sum|y|^2); columns with
// y = 0 count as converged when r = 0
__global__ void k_residual_ratio(const double* __restrict__ part, int njobs, int nchunk,
                                 const ResJob* __restrict__ jobs, double* __restrict__ ratio) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  double mx = 0.0;
  for (int c = 0; c < jobs[j].ncol; ++c) {
    double rr = 0.0, yy = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) {
      size_t o = (((size_t)j * nchunk + ch) * 32 + c) * 2;
      rr += part[o];
      yy += part[o + 1];
    }
    double q = yy > 0.0 ? sqrt(rr / yy) : (rr > 0.0 ? 1e300 : 0.0);
    if (!(q <= mx)) mx = q;  // NaN propagates
  }
  ratio[j] = mx;
}

size_t residual_part_doubles(int64_t n, int njobs) {
  int nchunk = (int)((n + kResChunk - 1) / kResChunk);
  return (size_t)njobs * nchunk * 32 * 2;
}

int launch_residual_jobs(const Band& bd, int njobs, const ResJob* jobs_dev, double* part,
                         double* ratio_dev, double work, hipStream_t st) {
  if (njobs <= 0) return 0;
  ProfScope ps(FB_PROF_RESID, st, work);
  int nchunk = (int)((bd.n + kResChunk - 1) / kResChunk);
  for (int j0 = 0; j0 < njobs; j0 += 65535) {
    int nj = njobs - j0 < 65535 ? njobs - j0 : 65535;
    dim3 grid(nchunk, nj);
    k_shift_residual<<<grid, 256, 0, st>>>(bd.Bd, bd.n, bd.b, jobs_dev + j0,
                                           part + (size_t)j0 * nchunk * 64, nchunk);
    FB_HIP(hipGetLastError());
  }
  k_residual_ratio<<<(njobs + 255) / 256, 256, 0, st>>>(part, njobs, nchunk, jobs_dev, ratio_dev);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
