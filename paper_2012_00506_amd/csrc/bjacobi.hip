// Parallel two-sided block Jacobi for the reduced Hermitian eigenproblems of
// the Rayleigh-Ritz step (Algorithm alg:FEAST: A_q W = W Lambda) and the
// Gram matrices of the eigen-decomposition orthonormalisation, for matrices
// too large for the one-workgroup Jacobi.
//
// The matrix is padded to mp = 64 h columns (the padding decoupled with a
// huge diagonal, so that it sorts last and is never rotated) and split into
// 2h blocks of 32 columns.  Blocks are kept in a physical order in which
// round r pairs positions (2k, 2k+1): one round
//  1. diagonalises every 64 x 64 principal block A[K, K] of pair K by a
//     cyclic Jacobi in LDS, giving a unitary U_K (k_bj_pairs);
//  2. forms A[K, L] <- U_K^H A[K, L] U_L for every pair of pairs and
//     V[:, L] <- V[:, L] U_L as two 64 x 64 x 64 complex products on FP64
//     MFMA per tile (k_bj_update), writing every 32-row/column block to its
//     position for the next round.
// Positions move between rounds as in the round-robin (circle) schedule:
// position 0 stays, the others advance one step around the ring
// 2, 4, ..., 2h-2, 2h-1, 2h-3, ..., 3, 1, so that over 2h - 1 rounds every
// two blocks share a pair once (one sweep).  Sweeps repeat until the
// off-diagonal part of A is below tol times its norm.
#include <math.h>

#include <algorithm>
#include <vector>

#include "prof.h"
#include "rr.h"

namespace fb {

static constexpr int kBs = 32;        // columns per block
static constexpr int kPb = 2 * kBs;   // columns per pair
static constexpr int kPL = kPb + 1;   // padded column length in LDS
static constexpr double kPad = 1e20;  // diagonal of the padding

struct BJDev {  // kBjDescBytes bytes
  c128* A[2];   // mp x mp, ld = mp (current / next)
  c128* V[2];   // mp x mp
  c128* U;      // h x 64 x 64, row-major per pair: U[K][k * 64 + j] = U_K(k, j)
  int32_t* skip;// h: U of the pair is the identity
  double* part; // 2 doubles per column of A: off^2 and total^2 partial sums
  int32_t m, mp, h, cur;
};

typedef double bd4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bd4 bj_mfma(double a, double b, bd4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// position of a block's content in the next round
__device__ __forceinline__ int bj_next(int pos, int h) {
  if (h == 1 || pos == 0) return pos;
  if ((pos & 1) == 0) {                       // top row, k = pos / 2 >= 1
    const int k = pos >> 1;
    return k < h - 1 ? pos + 2 : pos + 1;     // last top goes to the last bottom
  }
  const int k = pos >> 1;                     // bottom row
  return k >= 1 ? pos - 2 : 2;                // first bottom goes to top 1
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
    gst(d.A[0] + e, a);
    gst(d.V[0] + e, mk(i == j ? 1.0 : 0.0, 0.0));
  }
}

// -------------------------------------------------------------- off-norm
// padding columns and rows (diagonal kPad) are left out
__global__ void __launch_bounds__(256) k_bj_norms(BJDev* __restrict__ dv) {
  const BJDev d = dv[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= d.mp) return;
  const c128* A = (d.cur ? d.A[1] : d.A[0]);
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  const bool padj = gld(A + (int64_t)j * d.mp + j).x > 0.5 * kPad;
  if (!padj) {
    for (int i = threadIdx.x; i < d.mp; i += blockDim.x) {
      if (gld(A + (int64_t)i * d.mp + i).x > 0.5 * kPad) continue;
      double a = cabs2(gld(A + (int64_t)j * d.mp + i));
      all += a;
      if (i != j) off += a;
    }
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
  for (int j = 0; j < d.mp; ++j) {
    off += gld(d.part + 2 * j);
    all += gld(d.part + 2 * j + 1);
  }
  out[2 * q] = off;
  out[2 * q + 1] = all;
}

// -------------------------------------------------------------- pair solves
// One workgroup per (pair, matrix): one cyclic Jacobi sweep on the 64 x 64
// principal block (none once it is diagonal), accumulating U.  A second inner
// sweep makes U more exact but buys few outer sweeps: on the benchmark's
// reduced matrices (m = 1 346..1 551) one inner sweep took 43 outer sweeps
// against 40 in 1.9 s against 2.3 s.
static constexpr int kInner = 1;
static constexpr int kPairThreads = 1024;  // one 2 x 2 block update per thread per round

__device__ __forceinline__ int bj_player(int pos, int r, int n) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n - 1);
}

__global__ void __launch_bounds__(kPairThreads) k_bj_pairs(BJDev* __restrict__ dv) {
  extern __shared__ __align__(16) char lds_raw[];
  c128* S = reinterpret_cast<c128*>(lds_raw);  // column-major, ld kPL
  c128* Us = S + kPb * kPL;                    // column-major, ld kPL
  __shared__ double s_cs[kBs], s_sn[kBs];
  __shared__ c128 s_e[kBs];
  __shared__ int s_p[kBs], s_q[kBs];
  __shared__ double red[2][kPairThreads];
  const BJDev d = dv[blockIdx.y];
  const int K = blockIdx.x;
  if (K >= d.h) return;
  const int t = threadIdx.x;
  const c128* A = (d.cur ? d.A[1] : d.A[0]);
  const int64_t base = (int64_t)K * kPb;
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int cj = e / kPb, ci = e % kPb;
    S[cj * kPL + ci] = gld(A + (base + cj) * d.mp + base + ci);
    Us[cj * kPL + ci] = mk(ci == cj ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int rotated = 0;
  for (int sw = 0; sw < kInner; ++sw) {
    // stop when the block is diagonal relative to its (non-padding) diagonal
    double off = 0.0, dg = 0.0;
    for (int e = t; e < kPb * kPb; e += blockDim.x) {
      const int cj = e / kPb, ci = e % kPb;
      const c128 v = S[cj * kPL + ci];
      if (ci != cj) off += cabs2(v);
      else dg += fabs(v.x) < 0.5 * kPad ? cabs2(v) : 0.0;
    }
    red[0][t] = off;
    red[1][t] = dg;
    __syncthreads();
    for (int s = kPairThreads / 2; s > 0; s >>= 1) {
      if (t < s) {
        red[0][t] += red[0][t + s];
        red[1][t] += red[1][t + s];
      }
      __syncthreads();
    }
    const bool diag = !(red[0][0] > 1e-32 * red[1][0]);
    __syncthreads();
    if (diag) break;  // uniform: every thread read the same sums
    rotated = 1;
    for (int ro = 0; ro < kPb - 1; ++ro) {
      if (t < kBs) {
        const int a = bj_player(t, ro, kPb), b = bj_player(kPb - 1 - t, ro, kPb);
        const int p = a < b ? a : b, q = a < b ? b : a;
        s_p[t] = p;
        s_q[t] = q;
        double cs = 1.0, sn = 0.0;
        c128 e = mk(1.0, 0.0);
        const c128 c = S[q * kPL + p];
        const double ac = sqrt(cabs2(c));
        const double app = S[p * kPL + p].x, aqq = S[q * kPL + q].x;
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
      // S <- J^H S J by 2 x 2 blocks (pair kk rows, pair ll columns)
      for (int e2 = t; e2 < kBs * kBs; e2 += blockDim.x) {
        const int kk = e2 % kBs, ll = e2 / kBs;
        const int pk = s_p[kk], qk = s_q[kk], pl = s_p[ll], ql = s_q[ll];
        const c128 a00 = S[pl * kPL + pk], a10 = S[pl * kPL + qk];
        const c128 a01 = S[ql * kPL + pk], a11 = S[ql * kPL + qk];
        const double cl = s_cs[ll], sl = s_sn[ll];
        const c128 el = s_e[ll];
        const c128 b00 = cl * a00 - sl * (el * a01), b01 = sl * a00 + cl * (el * a01);
        const c128 b10 = cl * a10 - sl * (el * a11), b11 = sl * a10 + cl * (el * a11);
        const double ck = s_cs[kk], sk = s_sn[kk];
        const c128 ek = cconj(s_e[kk]);
        S[pl * kPL + pk] = ck * b00 - sk * (ek * b10);
        S[pl * kPL + qk] = sk * b00 + ck * (ek * b10);
        S[ql * kPL + pk] = ck * b01 - sk * (ek * b11);
        S[ql * kPL + qk] = sk * b01 + ck * (ek * b11);
      }
      // U <- U J (columns p, q)
      for (int e2 = t; e2 < kBs * kPb; e2 += blockDim.x) {
        const int kk = e2 / kPb, i = e2 % kPb;
        const int p = s_p[kk], q = s_q[kk];
        const double cs = s_cs[kk], sn = s_sn[kk];
        const c128 e = s_e[kk];
        const c128 vp = Us[p * kPL + i], vq = Us[q * kPL + i];
        Us[p * kPL + i] = cs * vp - sn * (e * vq);
        Us[q * kPL + i] = sn * vp + cs * (e * vq);
      }
      __syncthreads();
    }
  }
  c128* U = d.U + (size_t)K * kPb * kPb;
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int k = e / kPb, j = e % kPb;  // row-major
    gst(U + e, Us[j * kPL + k]);
  }
  if (t == 0) gst(d.skip + K, rotated ? 0 : 1);
}

// -------------------------------------------------------------- updates
// Workgroups 0 .. h(h+1)/2-1 of a matrix: the tiles (K, L), K <= L, of A,
// R = U_K^H A[K,L] U_L (R^H is the tile (L, K): A stays Hermitian);
// workgroups from h(h+1)/2 on: the tiles (I, L) of V, V[I, L] U_L.  Each
// 32-row and 32-column block of the result is written to its next-round
// position.  Four waves each own a 32 x 32 quarter of a 64 x 64 x 64
// product (2 x 2 MFMA tiles of 16 x 16, Gauss form); operand fragments are
// loaded one contraction step ahead.
template <bool CONJA, typename FA, typename FB>
__device__ __forceinline__ void bj_quarter(bd4 (&p1)[2][2], bd4 (&p2)[2][2], bd4 (&p3)[2][2],
                                           FA fa, FB fb, int lk) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) p1[a][b][r] = p2[a][b][r] = p3[a][b][r] = 0.0;
  c128 an[2], bn[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    an[q] = fa(q, lk);
    bn[q] = fb(q, lk);
  }
#pragma unroll 2
  for (int kk = 0; kk < kPb; kk += 4) {
    c128 ac[2] = {an[0], an[1]}, bc[2] = {bn[0], bn[1]};
    if (kk + 4 < kPb) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        an[q] = fa(q, kk + 4 + lk);
        bn[q] = fb(q, kk + 4 + lk);
      }
    }
    double ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ar[q] = ac[q].x;
      ai[q] = CONJA ? -ac[q].y : ac[q].y;
      as[q] = ar[q] + ai[q];
      br[q] = bc[q].x;
      bi[q] = bc[q].y;
      bs[q] = bc[q].x + bc[q].y;
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        p1[rt][ct] = bj_mfma(ar[rt], br[ct], p1[rt][ct]);
        p2[rt][ct] = bj_mfma(ai[rt], bi[ct], p2[rt][ct]);
        p3[rt][ct] = bj_mfma(as[rt], bs[ct], p3[rt][ct]);
      }
  }
}

__global__ void __launch_bounds__(256) k_bj_update(BJDev* __restrict__ dv) {
  extern __shared__ __align__(16) char lds_raw[];
  c128* Ts = reinterpret_cast<c128*>(lds_raw);  // 64 x 64, column-major, ld kPL
  const BJDev d = dv[blockIdx.y];
  const int h = d.h;
  const int nA = h * (h + 1) / 2, nV = h * (d.mp / kPb);
  const int wg = blockIdx.x;
  if (wg >= nA + nV) return;
  const bool isA = wg < nA;
  int K, L;
  if (isA) {  // wg -> (K, L), K <= L, row by row
    K = 0;
    int off = 0;
    while (off + (h - K) <= wg) {
      off += h - K;
      ++K;
    }
    L = K + (wg - off);
  } else {
    K = (wg - nA) / h;  // row tile of V
    L = (wg - nA) % h;
  }
  const int cur = d.cur;
  // (selects, not indexing: an indexed member array would live in scratch)
  const c128* Src = isA ? (cur ? d.A[1] : d.A[0]) : (cur ? d.V[1] : d.V[0]);
  c128* Dst = isA ? (cur ? d.A[0] : d.A[1]) : (cur ? d.V[0] : d.V[1]);
  const int64_t ld = d.mp;
  const int64_t r0 = (int64_t)K * kPb, c0 = (int64_t)L * kPb;
  const int skK = isA ? gld(d.skip + K) : 1, skL = gld(d.skip + L);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w & 1, wc = w >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const c128* UL = d.U + (size_t)L * kPb * kPb;
  const c128* UK = d.U + (size_t)K * kPb * kPb;
  bd4 p1[2][2], p2[2][2], p3[2][2];
  auto to_lds = [&]() {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 32 * wr + 16 * rt + lk + 4 * r, j = 32 * wc + 16 * ct + li;
          const double x1 = p1[rt][ct][r], x2 = p2[rt][ct][r], x3 = p3[rt][ct][r];
          Ts[j * kPL + i] = mk(x1 - x2, x3 - x1 - x2);
        }
  };

  if (skL) {  // no product on the right: the tile itself
    for (int e = t; e < kPb * kPb; e += blockDim.x) {
      const int j = e / kPb, i = e % kPb;
      Ts[j * kPL + i] = gld(Src + (c0 + j) * ld + r0 + i);
    }
  } else {  // T = Src[K, L] U_L
    bj_quarter<false>(
        p1, p2, p3,
        [&](int q, int k) { return gld(Src + (c0 + k) * ld + r0 + 32 * wr + 16 * q + li); },
        [&](int q, int k) { return gld(UL + k * kPb + 32 * wc + 16 * q + li); }, lk);
    to_lds();
  }
  __syncthreads();
  if (!skK) {  // R = U_K^H T
    bj_quarter<true>(
        p1, p2, p3, [&](int q, int k) { return gld(UK + k * kPb + 32 * wr + 16 * q + li); },
        [&](int q, int k) { return Ts[(32 * wc + 16 * q + li) * kPL + k]; }, lk);
    __syncthreads();  // every wave has read T
    to_lds();
    __syncthreads();
  }
  // write out: rows of an A tile move with their blocks, V rows stay; an
  // off-diagonal A tile also gives its conjugate transpose
  for (int e = t; e < kPb * kPb; e += blockDim.x) {
    const int j = e / kPb, i = e % kPb;
    const int64_t gr = isA ? (int64_t)bj_next(2 * K + i / kBs, h) * kBs + i % kBs : r0 + i;
    const int64_t gc = (int64_t)bj_next(2 * L + j / kBs, h) * kBs + j % kBs;
    gst(Dst + gc * ld + gr, Ts[j * kPL + i]);
  }
  if (isA && K != L) {
    for (int e = t; e < kPb * kPb; e += blockDim.x) {
      const int i = e / kPb, j = e % kPb;  // conj(R(i, j)) goes to (row of j, column of i)
      const int64_t gr = (int64_t)bj_next(2 * L + j / kBs, h) * kBs + j % kBs;
      const int64_t gc = (int64_t)bj_next(2 * K + i / kBs, h) * kBs + i % kBs;
      gst(Dst + gc * ld + gr, cconj(Ts[j * kPL + i]));
    }
  }
}

// -------------------------------------------------------------- results
// eigenvalues ascending (rank by value, ties by position; the padding ranks
// last) and the matching columns of V (first m rows) into the job's outputs
__global__ void k_bj_rank(const JacobiJob* __restrict__ jobs, BJDev* __restrict__ dv) {
  const JacobiJob jb = jobs[blockIdx.y];
  const BJDev d = dv[blockIdx.y];
  const c128* A = (d.cur ? d.A[1] : d.A[0]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.mp) return;
  const double wi = gld(A + (int64_t)i * d.mp + i).x;
  int rank = 0;
  for (int j = 0; j < d.mp; ++j) {
    const double wj = gld(A + (int64_t)j * d.mp + j).x;
    rank += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
  }
  if (rank < d.m) {
    gst(jb.w + rank, wi);
    gst(jb.order + rank, i);
  }
}

__global__ void k_bj_vectors(const JacobiJob* __restrict__ jobs, BJDev* __restrict__ dv) {
  const JacobiJob jb = jobs[blockIdx.y];
  const BJDev d = dv[blockIdx.y];
  const c128* V = (d.cur ? d.V[1] : d.V[0]);
  const int64_t tot = (int64_t)d.m * d.m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / d.m), i = (int)(e - (int64_t)k * d.m);
    const int src = gld(jb.order + k);
    gst(jb.W + (int64_t)k * jb.ldw + i, gld(V + (int64_t)src * d.mp + i));
  }
}

__global__ void k_bj_flip(BJDev* __restrict__ dv, int nmat) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nmat) dv[q].cur ^= 1;
}

// -------------------------------------------------------------- driver
static int bj_h(int m) { return (m + kPb - 1) / kPb; }

size_t block_jacobi_bytes(int m) {
  const int h = bj_h(m), mp = kPb * h;
  const size_t sq = ((size_t)mp * mp * sizeof(c128) + 255) & ~(size_t)255;
  return 4 * sq + (size_t)h * kPb * kPb * sizeof(c128) + 256 + (size_t)h * sizeof(int32_t) +
         256 + 2 * (size_t)mp * sizeof(double) + 4 * 256;
}

int block_jacobi(const std::vector<JacobiJob>& jobs, const JacobiJob* jobs_dev, char* work,
                 void* dv_dev, double* norms_dev, int max_sweeps, double tol, hipStream_t st) {
  const int nj = (int)jobs.size();
  if (nj == 0) return 0;
  std::vector<BJDev> dv(nj);
  int max_h = 0, max_mp = 0, max_rounds = 1;
  size_t off = 0;
  for (int q = 0; q < nj; ++q) {
    BJDev& d = dv[q];
    d.m = jobs[q].m;
    d.h = bj_h(d.m);
    d.mp = kPb * d.h;
    d.cur = 0;
    auto take = [&](size_t bytes) {
      char* p = work + off;
      off += (bytes + 255) & ~(size_t)255;
      return p;
    };
    const size_t sq = (size_t)d.mp * d.mp * sizeof(c128);
    d.A[0] = (c128*)take(sq);
    d.A[1] = (c128*)take(sq);
    d.V[0] = (c128*)take(sq);
    d.V[1] = (c128*)take(sq);
    d.U = (c128*)take((size_t)d.h * kPb * kPb * sizeof(c128));
    d.skip = (int32_t*)take((size_t)d.h * sizeof(int32_t));
    d.part = (double*)take(2 * (size_t)d.mp * sizeof(double));
    max_h = std::max(max_h, d.h);
    max_mp = std::max(max_mp, d.mp);
    max_rounds = std::max(max_rounds, 2 * d.h - 1);
  }
  static bool attr = false;
  const size_t lds_pairs = 2 * (size_t)kPb * kPL * sizeof(c128);
  const size_t lds_upd = (size_t)kPb * kPL * sizeof(c128);
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_bj_pairs, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_pairs);
    (void)hipFuncSetAttribute((const void*)k_bj_update, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_upd);
    (void)hipGetLastError();
    attr = true;
  }
  BJDev* dvd = (BJDev*)dv_dev;
  FB_HIP(hipMemcpyAsync(dvd, dv.data(), sizeof(BJDev) * nj, hipMemcpyHostToDevice, st));
  k_bj_init<<<dim3(1024, nj), 256, 0, st>>>(jobs_dev, dvd);
  FB_HIP(hipGetLastError());
  std::vector<double> nrm(2 * nj);
  int sweeps = 0;
  const int upd_wgs = max_h * (max_h + 1) / 2 + max_h * (max_mp / kPb);
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    k_bj_norms<<<dim3(max_mp, nj), 256, 0, st>>>(dvd);
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
    // every matrix takes max_rounds rounds (a smaller one completes further
    // sweeps of its own schedule, which keeps it converging)
    for (int r = 0; r < max_rounds; ++r) {
      k_bj_pairs<<<dim3(max_h, nj), kPairThreads, lds_pairs, st>>>(dvd);
      FB_HIP(hipGetLastError());
      k_bj_update<<<dim3(upd_wgs, nj), 256, lds_upd, st>>>(dvd);
      FB_HIP(hipGetLastError());
      k_bj_flip<<<(nj + 63) / 64, 64, 0, st>>>(dvd, nj);
      FB_HIP(hipGetLastError());
    }
  }
  k_bj_rank<<<dim3((max_mp + 255) / 256, nj), 256, 0, st>>>(jobs_dev, dvd);
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
