// Parallel two-sided block Jacobi for the reduced Hermitian eigenproblems of
// the Rayleigh-Ritz step and the orthonormalisation (Algorithm alg:FEAST:
// A_q W = W Lambda, and the Gram matrix Q^H Q), for matrices too large for
// the one-workgroup Jacobi.
//
// The padded matrix (mp = m rounded up to 32, padding decoupled with a huge
// diagonal so that it sorts last) is split into blocks of 16 columns.  One
// round pairs the blocks by the circle method; for every pair (I, J) the
// 32 x 32 principal submatrix A[K, K], K = I u J, is diagonalised by a
// cyclic Jacobi in LDS, giving a unitary U_K, and then
//   A[K, L] <- U_K^H A[K, L] U_L   for every pair of pairs (K, L),
//   V[:, L] <- V[:, L] U_L,
// each block of A and V written by exactly one workgroup.  Rounds repeat
// until the off-diagonal part of A is below tol times its norm (checked
// after every sweep of nb-1 rounds).
#include <math.h>

#include <algorithm>
#include <vector>

#include "prof.h"
#include "rr.h"

namespace fb {

static constexpr int kBs = 16;        // columns per block
static constexpr int kPb = 2 * kBs;   // columns per pair
static constexpr double kPad = 1e20;  // diagonal of the padding

struct BJDev {  // kBjDescBytes bytes
  c128* A;      // mp x mp, ld = mp
  c128* V;      // mp x mp
  c128* U;      // (nb/2) x kPb x kPb, column-major per pair
  int32_t* skip;// nb/2: U of the pair is the identity
  double* part; // 2 doubles per column of A: off^2 and total^2 partial sums
  int32_t m, mp, nb, pad_;
};

// player at position pos in round r (circle method, position 0 fixed)
__device__ __forceinline__ int bj_player(int pos, int r, int nb) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (nb - 1);
}

// global row/column index of entry e (0..31) of pair k in round r
__device__ __forceinline__ int bj_index(int k, int e, int r, int nb) {
  int a = bj_player(k, r, nb), b = bj_player(nb - 1 - k, r, nb);
  int lo = a < b ? a : b, hi = a < b ? b : a;
  return e < kBs ? lo * kBs + e : hi * kBs + (e - kBs);
}

// -------------------------------------------------------------- pad / init
__global__ void k_bj_init(const JacobiJob* __restrict__ jobs, BJDev* __restrict__ dv) {
  const JacobiJob jb = jobs[blockIdx.y];
  const BJDev d = dv[blockIdx.y];
  const int64_t tot = (int64_t)d.mp * d.mp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / d.mp), i = (int)(e - (int64_t)j * d.mp);
    c128 a = mk(0.0, 0.0);
    if (i < d.m && j < d.m)
      a = gld(jb.A + (int64_t)j * jb.lda + i);
    else if (i == j)
      a = mk(kPad, 0.0);
    gst(d.A + e, a);
    gst(d.V + e, mk(i == j ? 1.0 : 0.0, 0.0));
  }
}

// -------------------------------------------------------------- off-norm
__global__ void __launch_bounds__(256) k_bj_norms(BJDev* __restrict__ dv) {
  const BJDev d = dv[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= d.m) return;
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  for (int i = threadIdx.x; i < d.m; i += blockDim.x) {
    double a = cabs2(gld(d.A + (int64_t)j * d.mp + i));
    all += a;
    if (i != j) off += a;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    gst(d.part + 2 * j, r0[0]);
    gst(d.part + 2 * j + 1, r1[0]);
  }
}

__global__ void k_bj_norms_final(BJDev* __restrict__ dv, int nmat, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nmat) return;
  const BJDev d = dv[q];
  double off = 0.0, all = 0.0;
  for (int j = 0; j < d.m; ++j) {
    off += gld(d.part + 2 * j);
    all += gld(d.part + 2 * j + 1);
  }
  out[2 * q] = off;
  out[2 * q + 1] = all;
}

// -------------------------------------------------------------- pair solves
// One workgroup per (pair, matrix): cyclic Jacobi on the 32 x 32 principal
// submatrix (at most kInner sweeps), accumulating U.
static constexpr int kInner = 3;

__global__ void __launch_bounds__(256) k_bj_pairs(BJDev* __restrict__ dv, int r) {
  __shared__ c128 S[kPb * kPb];  // column-major
  __shared__ c128 Us[kPb * kPb];
  __shared__ double s_cs[kBs], s_sn[kBs];
  __shared__ c128 s_e[kBs];
  __shared__ int s_p[kBs], s_q[kBs];
  __shared__ double red[256];
  const BJDev d = dv[blockIdx.y];
  const int np = d.nb / 2;
  const int k = blockIdx.x;
  if (k >= np) return;
  const int t = threadIdx.x;
  const int rr = r % (d.nb - 1);
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int cj = e / kPb, ci = e % kPb;
    const int gi = bj_index(k, ci, rr, d.nb), gj = bj_index(k, cj, rr, d.nb);
    S[e] = gld(d.A + (int64_t)gj * d.mp + gi);
    Us[e] = mk(ci == cj ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // is the pair already diagonal (relative to its diagonal)?
  {
    double off = 0.0, dg = 0.0;
    for (int e = t; e < kPb * kPb; e += blockDim.x) {
      const int cj = e / kPb, ci = e % kPb;
      double a = cabs2(S[e]);
      if (ci != cj) off += a; else dg += (fabs(S[e].x) < 1e19 ? a : 0.0);
    }
    red[t] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[t] = dg;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    const double dgs = red[0];
    __syncthreads();
    if (!(offs > 1e-32 * dgs)) {
      if (t == 0) gst(d.skip + k, 1);
      return;  // uniform: every thread took the same branch
    }
  }
  for (int sw = 0; sw < kInner; ++sw) {
    for (int ro = 0; ro < kPb - 1; ++ro) {
      if (t < kBs) {
        const int a = bj_player(t, ro, kPb), b = bj_player(kPb - 1 - t, ro, kPb);
        const int p = a < b ? a : b, q = a < b ? b : a;
        s_p[t] = p;
        s_q[t] = q;
        double cs = 1.0, sn = 0.0;
        c128 e = mk(1.0, 0.0);
        const c128 c = S[q * kPb + p];
        const double ac = sqrt(cabs2(c));
        const double app = S[p * kPb + p].x, aqq = S[q * kPb + q].x;
        if (ac > 1e-300 && ac > 1e-18 * (fabs(app) + fabs(aqq))) {
          const double tau = (aqq - app) / (2.0 * ac);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
          cs = 1.0 / sqrt(1.0 + tt * tt);
          sn = tt * cs;
          e = mk(c.x / ac, -c.y / ac);  // e^{-i arg c}
        }
        s_cs[t] = cs;
        s_sn[t] = sn;
        s_e[t] = e;
      }
      __syncthreads();
      {
        // S <- J^H S J by 2 x 2 blocks (pair kk rows, pair ll columns)
        const int kk = t % kBs, ll = t / kBs;
        const int pk = s_p[kk], qk = s_q[kk], pl = s_p[ll], ql = s_q[ll];
        const c128 a00 = S[pl * kPb + pk], a10 = S[pl * kPb + qk];
        const c128 a01 = S[ql * kPb + pk], a11 = S[ql * kPb + qk];
        const double cl = s_cs[ll], sl = s_sn[ll];
        const c128 el = s_e[ll];
        const c128 b00 = cl * a00 - sl * (el * a01), b01 = sl * a00 + cl * (el * a01);
        const c128 b10 = cl * a10 - sl * (el * a11), b11 = sl * a10 + cl * (el * a11);
        const double ck = s_cs[kk], sk = s_sn[kk];
        const c128 ek = cconj(s_e[kk]);
        S[pl * kPb + pk] = ck * b00 - sk * (ek * b10);
        S[pl * kPb + qk] = sk * b00 + ck * (ek * b10);
        S[ql * kPb + pk] = ck * b01 - sk * (ek * b11);
        S[ql * kPb + qk] = sk * b01 + ck * (ek * b11);
      }
      // U <- U J (columns p, q)
      for (int e2 = t; e2 < kBs * kPb; e2 += blockDim.x) {
        const int kk = e2 / kPb, i = e2 % kPb;
        const int p = s_p[kk], q = s_q[kk];
        const double cs = s_cs[kk], sn = s_sn[kk];
        const c128 e = s_e[kk];
        const c128 vp = Us[p * kPb + i], vq = Us[q * kPb + i];
        Us[p * kPb + i] = cs * vp - sn * (e * vq);
        Us[q * kPb + i] = sn * vp + cs * (e * vq);
      }
      __syncthreads();
    }
  }
  c128* U = d.U + (size_t)k * kPb * kPb;
  for (int e = t; e < kPb * kPb; e += blockDim.x) gst(U + e, Us[e]);
  if (t == 0) gst(d.skip + k, 0);
}

// -------------------------------------------------------------- updates
// A[K, L] <- U_K^H A[K, L] U_L, one workgroup per (K, L, matrix)
__global__ void __launch_bounds__(256) k_bj_update_a(BJDev* __restrict__ dv, int r) {
  __shared__ c128 Ab[kPb * kPb];   // column-major block, then U_K^H (A U_L)
  __shared__ c128 T[kPb * kPb];
  __shared__ c128 Ul[kPb * kPb];   // column-major
  __shared__ c128 UkT[kPb * kPb];  // UkT[row * kPb + col] = U_K[row][col]: row-major
  const BJDev d = dv[blockIdx.z];
  const int np = d.nb / 2;
  const int kb = blockIdx.x, lb = blockIdx.y;
  if (kb >= np || lb >= np) return;
  const int skk = gld(d.skip + kb), skl = gld(d.skip + lb);
  if (skk && skl) return;
  const int t = threadIdx.x;
  const int rr = r % (d.nb - 1);
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int cj = e / kPb, ci = e % kPb;
    const int gi = bj_index(kb, ci, rr, d.nb), gj = bj_index(lb, cj, rr, d.nb);
    Ab[e] = gld(d.A + (int64_t)gj * d.mp + gi);
    Ul[e] = skl ? mk(ci == cj ? 1.0 : 0.0, 0.0) : gld(d.U + (size_t)lb * kPb * kPb + e);
    // U_K entry (row ci, col cj) stored row-major for the U^H product
    UkT[ci * kPb + cj] = skk ? mk(ci == cj ? 1.0 : 0.0, 0.0) : gld(d.U + (size_t)kb * kPb * kPb + e);
  }
  __syncthreads();
  // T = Ab U_L: thread owns row i = t % 32, columns c = t / 32 + 8 q
  const int i = t % kPb, c0 = t / kPb;
  {
    c128 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = mk(0.0, 0.0);
    for (int kk = 0; kk < kPb; ++kk) {
      const c128 a = Ab[kk * kPb + i];
#pragma unroll
      for (int q = 0; q < 4; ++q) cmac(acc[q], a, Ul[(c0 + 8 * q) * kPb + kk]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) T[(c0 + 8 * q) * kPb + i] = acc[q];
  }
  __syncthreads();
  // R = U_K^H T: R[i][c] = sum_kk conj(U_K[kk][i]) T[kk][c]
  {
    c128 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = mk(0.0, 0.0);
    for (int kk = 0; kk < kPb; ++kk) {
      const c128 u = cconj(UkT[kk * kPb + i]);
#pragma unroll
      for (int q = 0; q < 4; ++q) cmac(acc[q], u, T[(c0 + 8 * q) * kPb + kk]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c0 + 8 * q;
      const int gi = bj_index(kb, i, rr, d.nb), gj = bj_index(lb, c, rr, d.nb);
      gst(d.A + (int64_t)gj * d.mp + gi, acc[q]);
    }
  }
}

// V[:, L] <- V[:, L] U_L, one workgroup per (32-row tile, L, matrix)
__global__ void __launch_bounds__(256) k_bj_update_v(BJDev* __restrict__ dv, int r) {
  __shared__ c128 Vb[kPb * kPb];
  __shared__ c128 Ul[kPb * kPb];
  const BJDev d = dv[blockIdx.z];
  const int np = d.nb / 2;
  const int lb = blockIdx.y, row0 = blockIdx.x * kPb;
  if (lb >= np || row0 >= d.mp) return;
  if (gld(d.skip + lb)) return;
  const int t = threadIdx.x;
  const int rr = r % (d.nb - 1);
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int cj = e / kPb, ci = e % kPb;
    const int gj = bj_index(lb, cj, rr, d.nb);
    Vb[e] = gld(d.V + (int64_t)gj * d.mp + row0 + ci);
    Ul[e] = gld(d.U + (size_t)lb * kPb * kPb + e);
  }
  __syncthreads();
  const int i = t % kPb, c0 = t / kPb;
  c128 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = mk(0.0, 0.0);
  for (int kk = 0; kk < kPb; ++kk) {
    const c128 a = Vb[kk * kPb + i];
#pragma unroll
    for (int q = 0; q < 4; ++q) cmac(acc[q], a, Ul[(c0 + 8 * q) * kPb + kk]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gj = bj_index(lb, c0 + 8 * q, rr, d.nb);
    gst(d.V + (int64_t)gj * d.mp + row0 + i, acc[q]);
  }
}

// -------------------------------------------------------------- results
// eigenvalues ascending (rank by value, ties by index) and the matching
// columns of V (first m rows) into the job's outputs
__global__ void k_bj_rank(const JacobiJob* __restrict__ jobs, BJDev* __restrict__ dv) {
  const JacobiJob jb = jobs[blockIdx.y];
  const BJDev d = dv[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  const double wi = gld(d.A + (int64_t)i * d.mp + i).x;
  int rank = 0;
  for (int j = 0; j < d.m; ++j) {
    const double wj = gld(d.A + (int64_t)j * d.mp + j).x;
    rank += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
  }
  gst(jb.w + rank, wi);
  gst(jb.order + rank, i);
}

__global__ void k_bj_vectors(const JacobiJob* __restrict__ jobs, BJDev* __restrict__ dv) {
  const JacobiJob jb = jobs[blockIdx.y];
  const BJDev d = dv[blockIdx.y];
  const int64_t tot = (int64_t)d.m * d.m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / d.m), i = (int)(e - (int64_t)k * d.m);
    const int src = gld(jb.order + k);
    gst(jb.W + (int64_t)k * jb.ldw + i, gld(d.V + (int64_t)src * d.mp + i));
  }
}

// -------------------------------------------------------------- driver
size_t block_jacobi_bytes(int m) {
  const int mp = (m + kPb - 1) / kPb * kPb;
  const int np = mp / kPb;
  return 2 * (size_t)mp * mp * sizeof(c128) + (size_t)np * kPb * kPb * sizeof(c128) +
         (size_t)np * sizeof(int32_t) + 2 * (size_t)mp * sizeof(double) + 4 * 256;
}

int block_jacobi(const std::vector<JacobiJob>& jobs, const JacobiJob* jobs_dev, char* work,
                 void* dv_dev, double* norms_dev, int max_sweeps, double tol, hipStream_t st) {
  const int nj = (int)jobs.size();
  if (nj == 0) return 0;
  std::vector<BJDev> dv(nj);
  int max_np = 0, max_mp = 0, max_m = 0, max_rounds = 1;
  size_t off = 0;
  for (int q = 0; q < nj; ++q) {
    BJDev& d = dv[q];
    d.m = jobs[q].m;
    d.mp = (d.m + kPb - 1) / kPb * kPb;
    d.nb = d.mp / kBs;
    const int np = d.nb / 2;
    auto take = [&](size_t bytes) {
      char* p = work + off;
      off += (bytes + 255) & ~(size_t)255;
      return p;
    };
    d.A = (c128*)take((size_t)d.mp * d.mp * sizeof(c128));
    d.V = (c128*)take((size_t)d.mp * d.mp * sizeof(c128));
    d.U = (c128*)take((size_t)np * kPb * kPb * sizeof(c128));
    d.skip = (int32_t*)take((size_t)np * sizeof(int32_t));
    d.part = (double*)take(2 * (size_t)d.mp * sizeof(double));
    max_np = std::max(max_np, np);
    max_mp = std::max(max_mp, d.mp);
    max_m = std::max(max_m, d.m);
    max_rounds = std::max(max_rounds, d.nb - 1);
  }
  BJDev* dvd = (BJDev*)dv_dev;
  FB_HIP(hipMemcpyAsync(dvd, dv.data(), sizeof(BJDev) * nj, hipMemcpyHostToDevice, st));
  k_bj_init<<<dim3(1024, nj), 256, 0, st>>>(jobs_dev, dvd);
  FB_HIP(hipGetLastError());
  std::vector<double> nrm(2 * nj);
  int sweeps = 0;
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    k_bj_norms<<<dim3(max_m, nj), 256, 0, st>>>(dvd);
    FB_HIP(hipGetLastError());
    k_bj_norms_final<<<(nj + 63) / 64, 64, 0, st>>>(dvd, nj, norms_dev);
    FB_HIP(hipGetLastError());
    FB_HIP(hipMemcpyAsync(nrm.data(), norms_dev, sizeof(double) * 2 * nj, hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    bool done = true;
    for (int q = 0; q < nj; ++q)
      if (!(nrm[2 * q] <= tol * tol * nrm[2 * q + 1])) done = false;
    if (done || sw == max_sweeps) break;
    ++sweeps;
    for (int r = 0; r < max_rounds; ++r) {
      k_bj_pairs<<<dim3(max_np, nj), 256, 0, st>>>(dvd, r);
      FB_HIP(hipGetLastError());
      k_bj_update_a<<<dim3(max_np, max_np, nj), 256, 0, st>>>(dvd, r);
      FB_HIP(hipGetLastError());
      k_bj_update_v<<<dim3(max_mp / kPb, max_np, nj), 256, 0, st>>>(dvd, r);
      FB_HIP(hipGetLastError());
    }
  }
  k_bj_rank<<<dim3((max_m + 255) / 256, nj), 256, 0, st>>>(jobs_dev, dvd);
  FB_HIP(hipGetLastError());
  k_bj_vectors<<<dim3(1024, nj), 256, 0, st>>>(jobs_dev, dvd);
  FB_HIP(hipGetLastError());
  for (int q = 0; q < nj; ++q)
    if (jobs[q].sweeps) FB_HIP(hipMemcpyAsync(jobs[q].sweeps, &sweeps, sizeof(int32_t),
                                              hipMemcpyHostToDevice, st));
  FB_HIP(hipStreamSynchronize(st));
  return 0;
}

static_assert(sizeof(BJDev) <= kBjDescBytes, "descriptor size");

size_t eig_work_bytes(const std::vector<int>& ms) {
  size_t b = 0;
  int n = 0;
  for (int m : ms)
    if (m > kSmallJacobi) {
      b += (block_jacobi_bytes(m) + 255) & ~(size_t)255;
      ++n;
    }
  return b + (size_t)n * kBjDescBytes + 2 * (size_t)n * sizeof(double) + 1024;
}

void carve_eig_work(Arena& ar, const std::vector<int>& ms, EigWork& w) {
  size_t b = 0;
  int n = 0;
  for (int m : ms)
    if (m > kSmallJacobi) {
      b += (block_jacobi_bytes(m) + 255) & ~(size_t)255;
      ++n;
    }
  w.bj = n ? ar.take<char>(b + 256 * (size_t)n) : nullptr;
  w.dv = n ? (void*)ar.take<char>((size_t)n * kBjDescBytes) : nullptr;
  w.norms = n ? ar.take<double>(2 * (size_t)n) : nullptr;
}

int reduced_eig(std::vector<JacobiJob> jobs, JacobiJob* jobs_dev, const EigWork& w,
                int max_sweeps, double tol, hipStream_t st) {
  std::vector<JacobiJob> small, large;
  for (const JacobiJob& j : jobs) (j.m > kSmallJacobi ? large : small).push_back(j);
  std::vector<JacobiJob> all(small);
  all.insert(all.end(), large.begin(), large.end());
  if (all.empty()) return 0;
  FB_HIP(hipMemcpyAsync(jobs_dev, all.data(), sizeof(JacobiJob) * all.size(),
                        hipMemcpyHostToDevice, st));
  if (!small.empty()) FB_TRY(launch_jacobi((int)small.size(), jobs_dev, max_sweeps, tol, st));
  if (!large.empty()) {
    if (!w.bj) return FB_ERR_INTERNAL;
    ProfScope ps(FB_PROF_JACOBI, st, 0.0);
    FB_TRY(block_jacobi(large, jobs_dev + small.size(), w.bj, w.dv, w.norms, max_sweeps, tol, st));
  }
  return 0;
}

}  // namespace fb
