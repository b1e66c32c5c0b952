// MFMA block-solve kernel templates (instantiated per precision in
// solve_f32.hip and solve_f64.hip).
#pragma once
#include "fb_internal.h"
#include "prof.h"
#include "solve_job.h"
#include "tune.h"

namespace fb {

// ---------------------------------------------------------------- MFMA helpers
// One wave computes a 16-row block of a complex product C (16 x T) +=
// A (16 x K rows of an NB x NB block) * B (K x T, in LDS), as three real
// 16x16x4 MFMAs per complex one (Gauss form, see Acc).  Lane l feeds
// A[l % 16][k + l / 16] and B[k + l / 16][l % 16].  Register r of lane l
// holds C[row][l % 16] with row = 4 (l / 16) + r for the f32 instruction and
// row = l / 16 + 4 r for the f64 one (both checked on gfx950).
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MF;
template <>
struct MF<float> {
  using V = mf_f4;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MF<double> {
  using V = mf_d4;
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Complex accumulator of NC 16 x 16 tiles in Gauss form: the value is
// (p1 - p2) + i (p3 - p1 - p2), so that a complex product takes three real
// MFMA products (p1 += Ar Br, p2 += Ai Bi, p3 += (Ar + Ai)(Br + Bi)).
template <typename R, int NC>
struct Acc {
  typename MF<R>::V p1[NC], p2[NC], p3[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        p1[c][r] = (R)0;
        p2[c][r] = (R)0;
        p3[c][r] = (R)0;
      }
  }
  __device__ __forceinline__ cx<R> get(int c, int r) const {
    return mk<R>(p1[c][r] - p2[c][r], p3[c][r] - p1[c][r] - p2[c][r]);
  }
  __device__ __forceinline__ void set(int c, int r, cx<R> v) {
    p1[c][r] = v.x;
    p2[c][r] = (R)0;
    p3[c][r] = v.x + v.y;
  }
};

// A fragments of one wave for one block product: register s holds
// op(A)[16 w + lane % 16][4 s + lane / 16] (complex), op(A) = A or A^H.
template <typename R, int NB>
struct Frag {
  cx<R> a[NB / 4];
};

// k ranges [k0, k1) are multiples of 16 and the same for the whole wave
// (readfirstlane makes that visible to the compiler, so that the range test
// is one scalar branch per 16-row chunk and a chunk's LDS reads issue
// together).  TS: A points at the transposed copy of the block (CONJT only),
// so that the 16 lanes of a fragment row read consecutive elements.
template <typename R, int NB, bool CONJT, typename PA, bool TS = false>
__device__ __forceinline__ void frag_load(Frag<R, NB>& f, PA A, int w, int lane, int k0, int k1) {
  const int i = 16 * w + (lane & 15), kq = lane >> 4;
  const int c0 = __builtin_amdgcn_readfirstlane(k0) >> 4;
  const int c1 = __builtin_amdgcn_readfirstlane(k1) >> 4;
#pragma unroll
  for (int ch = 0; ch < NB / 16; ++ch) {
    if (ch < c0 || ch >= c1) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 16 * ch + 4 * q + kq;
      f.a[4 * ch + q] = (CONJT && !TS) ? A[(size_t)i * NB + k] : A[(size_t)k * NB + i];
    }
  }
}

// acc += op(A) * B over k in [k0, k1) from prefetched fragments; NEG
// subtracts.  B row k is LDS row rmap[k] (or k when rmap is null), row
// stride ldb elements, columns from cb0.
template <typename R, int NB, int NC, bool CONJT, bool NEG>
__device__ __forceinline__ void frag_mma(Acc<R, NC>& acc, const Frag<R, NB>& f, const cx<R>* Bl,
                                         int ldb, const int* rmap, int cb0, int lane, int k0,
                                         int k1) {
  const int kq = lane >> 4;
  const int j = lane & 15;
  const int c0 = __builtin_amdgcn_readfirstlane(k0) >> 4;
  const int c1 = __builtin_amdgcn_readfirstlane(k1) >> 4;
#pragma unroll
  for (int ch = 0; ch < NB / 16; ++ch) {
    if (ch < c0 || ch >= c1) continue;
    cx<R> bv[4][NC];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 16 * ch + 4 * q + kq;
      const int br = rmap ? rmap[k] : k;
      const cx<R>* bp = Bl + (size_t)br * ldb + cb0 + j;
#pragma unroll
      for (int c = 0; c < NC; ++c) bv[q][c] = bp[16 * c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cx<R> a = f.a[4 * ch + q];
      R ar = a.x, ai = CONJT ? -a.y : a.y;
      if (NEG) {
        ar = -ar;
        ai = -ai;
      }
      const R as = ar + ai;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc.p1[c] = MF<R>::mma(ar, bv[q][c].x, acc.p1[c]);
        acc.p2[c] = MF<R>::mma(ai, bv[q][c].y, acc.p2[c]);
        acc.p3[c] = MF<R>::mma(as, bv[q][c].x + bv[q][c].y, acc.p3[c]);
      }
    }
  }
}

template <typename R, int NB, int NC, bool CONJT, bool NEG, typename PA>
__device__ __forceinline__ void wave_prod(Acc<R, NC>& acc, PA A, const cx<R>* Bl, int ldb,
                                          const int* rmap, int w, int cb0, int lane, int k0,
                                          int k1) {
  Frag<R, NB> f;
  frag_load<R, NB, CONJT>(f, A, w, lane, k0, k1);
  frag_mma<R, NB, NC, CONJT, NEG>(acc, f, Bl, ldb, rmap, cb0, lane, k0, k1);
}

// accumulator <-> LDS rows (rows 16 w + MF<R>::row(lane, r), columns 16 c + lane%16)
template <typename R, int NC>
__device__ __forceinline__ void acc_to_lds(const Acc<R, NC>& acc, cx<R>* L, int ldb,
                                           const int* rmap, int w, int cb0, int lane) {
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * w + MF<R>::row(lane, r);
      int lr = rmap ? rmap[row] : row;
      L[(size_t)lr * ldb + cb0 + 16 * c + (lane & 15)] = acc.get(c, r);
    }
}
template <typename R, int NC>
__device__ __forceinline__ void acc_from_lds(Acc<R, NC>& acc, const cx<R>* L, int ldb,
                                             const int* rmap, int w, int cb0, int lane) {
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * w + MF<R>::row(lane, r);
      int lr = rmap ? rmap[row] : row;
      acc.set(c, r, L[(size_t)lr * ldb + cb0 + 16 * c + (lane & 15)]);
    }
}

static __device__ __forceinline__ int remap_job(int bid, int njobs) {
  // consecutive jobs (one system's tiles) on one XCD: workgroups are dealt
  // to the 8 XCDs round-robin, so XCD x runs the x-th contiguous range
  const int per = (njobs + 7) / 8;
  return (bid % 8) * per + bid / 8;
}

// One block's initial accumulator values for a wave, raw (c128 for the
// right-hand sides, the factors' type for the intermediates), converted when
// first used so that the loads do not wait where they are issued.
template <typename E, int NC>
struct PreT {
  E v[NC][4];
  int k;
};

// ---------------------------------------------------------------- MFMA block solve
// One workgroup per job with one wave per 16 x (16 NC) output tile of a block
// product ((NB/16) x (T/(16 NC)) waves; a wave with NC > 1 reuses each factor
// fragment for NC column tiles); LDS holds 3 NB x T blocks.  OCC > 1 asks the
// compiler to fit the registers of OCC waves per SIMD.
template <typename R, int NB, int T, bool PREF, int NC, int OCC>
__global__ void __launch_bounds__(NB * 4 * (T / (16 * NC)), OCC)
k_band_solve(const cx<R>* __restrict__ mats, const cx<R>* __restrict__ matsT,
             const int16_t* __restrict__ permg, int64_t n, int K,
             const SolveJob* __restrict__ jobs, int njobs, const int32_t* __restrict__ gate) {
  // complex64 H solves read the transposed copy of the factor blocks
  constexpr bool TS = sizeof(R) == 4;
  constexpr int NRW = NB / 16;
  extern __shared__ __align__(16) char lds_raw[];
  int* sp = reinterpret_cast<int*>(lds_raw);                        // 2 NB perm entries
  cx<R>* S = reinterpret_cast<cx<R>*>(lds_raw + ((2 * NB * sizeof(int) + 15) & ~15));
  const int job = remap_job(blockIdx.x, njobs);
  if (job >= njobs) return;
  const SolveJob jb = jobs[job];
  if (gate && !gate[jb.grp]) return;  // a correction its group no longer needs
  const int t = threadIdx.x, lane = t & 63;
  // row block and column base of this wave (wave-uniform: scalar registers)
  const int w = __builtin_amdgcn_readfirstlane((t >> 6) % NRW);
  const int cb0 = __builtin_amdgcn_readfirstlane(16 * NC * ((t >> 6) / NRW));
  const int nthr = NB * 4 * (T / (16 * NC));
  const size_t bb = (size_t)NB * NB;
  const cx<R>* F = mats + (size_t)jb.sys * K * 5 * bb;
  const int16_t* P = permg + (size_t)jb.sys * K * 2 * NB;
  const c128* in = jb.in + (int64_t)jb.col0 * jb.ldin;
  cx<R>* mid = reinterpret_cast<cx<R>*>(jb.mid) + (int64_t)jb.col0 * jb.ldmid;
  c128* out = jb.out + (int64_t)jb.col0 * jb.ldout;
  const int ncol = jb.ncol;

  // Global loads are branch-free (an out-of-range element reads the tile's
  // first element and is zeroed when used), so that a group of loads issues
  // together and waits once, where its values are first needed.
  auto okf = [&](int64_t row, int col) { return row < n && col < ncol; };
  auto gaddr = [&](auto base, int64_t ld, int64_t row, int col) {
    return base + (okf(row, col) ? (int64_t)col * ld + row : 0);
  };
  auto conv = [&](auto v, bool ok) -> cx<R> {
    return ok ? mk<R>((R)v.x, (R)v.y) : mk<R>(0, 0);
  };
  // x into the output (added to it for a correction), a batch at a time:
  // all loads of the batch first, then the stores
  auto emit_batch = [&](auto& row, auto& col, auto& v, auto& valid) {
    constexpr int NQ = sizeof(valid) / sizeof(valid[0]);
    c128 old[NQ];
    if (jb.add) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) old[q] = gld(gaddr(out, jb.ldout, row[q], col[q]));
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (!valid[q] || !okf(row[q], col[q])) continue;
      c128 x = mk((double)v[q].x, (double)v[q].y);
      if (jb.add) x = old[q] + x;
      gst(out + (int64_t)col[q] * jb.ldout + row[q], x);
    }
  };
  constexpr int RE = 4 * NC;
  auto acc_to_g = [&](const Acc<R, NC>& acc, auto base, int64_t ld, int64_t row0) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t row = row0 + 16 * w + MF<R>::row(lane, r);
        int col = cb0 + 16 * c + (lane & 15);
        if (row < n && col < ncol)
          gst(base + (int64_t)col * ld + row, acc.get(c, r));
      }
  };
  auto acc_emit = [&](const Acc<R, NC>& acc, int64_t row0) {
    int64_t rows[RE];
    int cols[RE];
    cx<R> v[RE];
    bool valid[RE];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 4 * c + r;
        rows[q] = row0 + 16 * w + MF<R>::row(lane, r);
        cols[q] = cb0 + 16 * c + (lane & 15);
        v[q] = acc.get(c, r);
        valid[q] = true;
      }
    emit_batch(rows, cols, v, valid);
  };
  // a whole NB x T block of global rows (row0 ..) into LDS rows (dst)
  constexpr int NTHR = NB * 4 * (T / (16 * NC));
  constexpr int RF = NB * T / NTHR;  // elements per thread
  struct Fill {
    c128 v[RF];
  };
  auto fill_issue = [&](Fill& f, auto base, int64_t ld, int64_t row0) {
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      const int e = t + q * NTHR;
      f.v[q] = gld(gaddr(base, ld, row0 + e / T, e % T));
    }
  };
  auto fill_store = [&](const Fill& f, cx<R>* dst, int64_t row0) {
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      const int e = t + q * NTHR;
      dst[e] = conv(f.v[q], okf(row0 + e / T, e % T));
    }
  };
  auto load_perm = [&](int k) {
    for (int e = t; e < 2 * NB; e += nthr) sp[e] = gld(P + (size_t)k * 2 * NB + e);
  };
  // the permutation of block k fetched early into registers, stored later
  constexpr int RP = (2 * NB + NTHR - 1) / NTHR;
  struct PermPre {
    int16_t v[RP];
  };
  auto perm_issue = [&](PermPre& pp, int k) {
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      const int e = t + q * NTHR;
      pp.v[q] = gld(P + (size_t)k * 2 * NB + (e < 2 * NB ? e : 0));
    }
  };
  auto perm_store = [&](const PermPre& pp) {
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      const int e = t + q * NTHR;
      if (e < 2 * NB) sp[e] = pp.v[q];
    }
  };
  const int lo_tri = 16 * w + 16;  // k < lo_tri: lower triangle rows of this wave
  const int up_tri = 16 * w;       // k >= up_tri: upper triangle
  auto blk = [&](int k, int slot) { return F + ((size_t)k * 5 + slot) * bb; };
  const cx<R>* FT = TS ? matsT + (size_t)jb.sys * K * 5 * bb : F;
  auto blkh = [&](int k, int slot) { return FT + ((size_t)k * 5 + slot) * bb; };
  // initial accumulator values for the wave's rows of block k, prefetched
  // into registers one step ahead
  auto pre_load = [&](auto& p, auto base, int64_t ld, int k) {
    p.k = k;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        p.v[c][r] = gld(gaddr(base, ld, (int64_t)k * NB + 16 * w + MF<R>::row(lane, r),
                              cb0 + 16 * c + (lane & 15)));
  };
  auto pre_to_acc = [&](Acc<R, NC>& acc, const auto& p) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc.set(c, r, conv(p.v[c][r], okf((int64_t)p.k * NB + 16 * w + MF<R>::row(lane, r),
                                          cb0 + 16 * c + (lane & 15))));
      }
  };
  Acc<R, NC> acc;
  Frag<R, NB> fa, fb, fc;
  PreT<cx<R>, NC> pvm;  // intermediates (backward sweeps)
  PreT<c128, NC> pvi;   // right-hand sides (H forward)

  if (jb.dir == 0) {
    // ---------------------------------------------------------- N forward
    cx<R>* W = S;                 // window, 2 NB x T
    cx<R>* Yt = S + 2 * NB * T;   // y_top, NB x T
    {
      Fill f0, f1;
      fill_issue(f0, in, jb.ldin, 0);
      fill_issue(f1, in, jb.ldin, NB);
      fill_store(f0, W, 0);
      fill_store(f1, W + NB * T, NB);
    }
    Fill fr;
    load_perm(0);
    if (PREF) frag_load<R, NB, false>(fa, blk(0, 0), w, lane, 0, lo_tri);
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      if (PREF) frag_load<R, NB, false>(fb, blk(k, 1), w, lane, 0, NB);
      if (!PREF) frag_load<R, NB, false>(fa, blk(k, 0), w, lane, 0, lo_tri);
      acc.zero();
      frag_mma<R, NB, NC, false, false>(acc, fa, W, T, sp, cb0, lane, 0, lo_tri);
      acc_to_lds(acc, Yt, T, nullptr, w, cb0, lane);
      acc_to_g(acc, mid, jb.ldmid, (int64_t)k * NB);
      __syncthreads();
      fill_issue(fr, in, jb.ldin, (int64_t)(k + 2) * NB);  // consumed after the product
      PermPre pnext;
      if (k + 1 < K) perm_issue(pnext, k + 1);
      if (PREF && k + 1 < K) frag_load<R, NB, false>(fa, blk(k + 1, 0), w, lane, 0, lo_tri);
      if (!PREF) frag_load<R, NB, false>(fb, blk(k, 1), w, lane, 0, NB);
      acc_from_lds(acc, W, T, sp + NB, w, cb0, lane);
      frag_mma<R, NB, NC, false, true>(acc, fb, Yt, T, nullptr, cb0, lane, 0, NB);
      __syncthreads();
      acc_to_lds(acc, W, T, nullptr, w, cb0, lane);
      fill_store(fr, W + NB * T, (int64_t)(k + 2) * NB);
      if (k + 1 < K) perm_store(pnext);
      __syncthreads();
    }
    // ---------------------------------------------------------- N backward
    cx<R>* X1 = S;
    cx<R>* X2 = S + NB * T;
    cx<R>* V = S + 2 * NB * T;
    for (int e = t; e < 2 * NB * T; e += nthr) S[e] = mk<R>(0, 0);
    // fa = U(k,k+1), fb = U(k,k+2), fc = U(k,k)^{-1}, pv = y_k: prefetched
    if (PREF) frag_load<R, NB, false>(fc, blk(K - 1, 2), w, lane, up_tri, NB);
    pre_load(pvm, mid, jb.ldmid, K - 1);
    __syncthreads();
    for (int k = K - 1; k >= 0; --k) {
      if (!PREF && k + 1 < K) frag_load<R, NB, false>(fa, blk(k, 3), w, lane, 0, NB);
      if (!PREF && k + 2 < K) frag_load<R, NB, false>(fb, blk(k, 4), w, lane, 0, lo_tri);
      pre_to_acc(acc, pvm);
      if (k + 1 < K) frag_mma<R, NB, NC, false, true>(acc, fa, X1, T, nullptr, cb0, lane, 0, NB);
      if (k + 2 < K) frag_mma<R, NB, NC, false, true>(acc, fb, X2, T, nullptr, cb0, lane, 0, lo_tri);
      acc_to_lds(acc, V, T, nullptr, w, cb0, lane);
      __syncthreads();
      if (k > 0) {
        if (PREF && k < K) frag_load<R, NB, false>(fa, blk(k - 1, 3), w, lane, 0, NB);
        if (PREF && k + 1 < K) frag_load<R, NB, false>(fb, blk(k - 1, 4), w, lane, 0, lo_tri);
        pre_load(pvm, mid, jb.ldmid, k - 1);
      }
      if (!PREF) frag_load<R, NB, false>(fc, blk(k, 2), w, lane, up_tri, NB);
      acc.zero();
      frag_mma<R, NB, NC, false, false>(acc, fc, V, T, nullptr, cb0, lane, up_tri, NB);
      if (PREF && k > 0) frag_load<R, NB, false>(fc, blk(k - 1, 2), w, lane, up_tri, NB);
      acc_emit(acc, (int64_t)k * NB);
      acc_to_lds(acc, X2, T, nullptr, w, cb0, lane);
      __syncthreads();
      cx<R>* tmp = X1;
      X1 = X2;
      X2 = tmp;
    }
  } else {
    // ---------------------------------------------------------- H forward (U^H)
    cx<R>* W1 = S;
    cx<R>* W2 = S + NB * T;
    cx<R>* V = S + 2 * NB * T;
    for (int e = t; e < 2 * NB * T; e += nthr) S[e] = mk<R>(0, 0);
    // fa = U(k-1,k)^H, fb = U(k-2,k)^H, fc = U(k,k)^{-H}, pv = y_k
    if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(0, 2), w, lane, 0, lo_tri);
    pre_load(pvi, in, jb.ldin, 0);
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      if (!PREF && k >= 1) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k - 1, 3), w, lane, 0, NB);
      if (!PREF && k >= 2) frag_load<R, NB, true, const cx<R>*, TS>(fb, blkh(k - 2, 4), w, lane, up_tri, NB);
      pre_to_acc(acc, pvi);
      if (k >= 1) frag_mma<R, NB, NC, true, true>(acc, fa, W1, T, nullptr, cb0, lane, 0, NB);
      if (k >= 2) frag_mma<R, NB, NC, true, true>(acc, fb, W2, T, nullptr, cb0, lane, up_tri, NB);
      acc_to_lds(acc, V, T, nullptr, w, cb0, lane);
      __syncthreads();
      if (k + 1 < K) {
        if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k, 3), w, lane, 0, NB);
        if (PREF && k >= 1) frag_load<R, NB, true, const cx<R>*, TS>(fb, blkh(k - 1, 4), w, lane, up_tri, NB);
        pre_load(pvi, in, jb.ldin, k + 1);
      }
      if (!PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k, 2), w, lane, 0, lo_tri);
      acc.zero();
      frag_mma<R, NB, NC, true, false>(acc, fc, V, T, nullptr, cb0, lane, 0, lo_tri);
      if (PREF && k + 1 < K) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k + 1, 2), w, lane, 0, lo_tri);
      acc_to_g(acc, mid, jb.ldmid, (int64_t)k * NB);
      acc_to_lds(acc, W2, T, nullptr, w, cb0, lane);
      __syncthreads();
      cx<R>* tmp = W1;
      W1 = W2;
      W2 = tmp;
    }
    // ---------------------------------------------------------- H backward (L^H)
    // Three rotating blocks: the carry (window bottom), the L^H step's
    // intermediate and the window top.  The intermediate block is dead once
    // the window top is formed, so it receives the next carry, and the two
    // exchange roles for the next step.
    cx<R>* Vt = S;               // top of the window after the L^H step
    cx<R>* T1 = S + NB * T;      // intermediate, then the next carry
    cx<R>* Cb = S + 2 * NB * T;  // carry: window bottom
    for (int e = t; e < NB * T; e += nthr) Cb[e] = mk<R>(0, 0);
    load_perm(K - 1);
    // fa = Lh21^H, fc = (Lh11^{-1})^H, pv = w_k
    if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(K - 1, 1), w, lane, 0, NB);
    if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(K - 1, 0), w, lane, up_tri, NB);
    pre_load(pvm, mid, jb.ldmid, K - 1);
    __syncthreads();
    for (int k = K - 1; k >= 0; --k) {
      if (!PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k, 1), w, lane, 0, NB);
      pre_to_acc(acc, pvm);
      frag_mma<R, NB, NC, true, true>(acc, fa, Cb, T, nullptr, cb0, lane, 0, NB);
      acc_to_lds(acc, T1, T, nullptr, w, cb0, lane);
      __syncthreads();
      PermPre pnext;
      if (k > 0) {
        if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k - 1, 1), w, lane, 0, NB);
        pre_load(pvm, mid, jb.ldmid, k - 1);
        perm_issue(pnext, k - 1);
      }
      if (!PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k, 0), w, lane, up_tri, NB);
      acc.zero();
      frag_mma<R, NB, NC, true, false>(acc, fc, T1, T, nullptr, cb0, lane, up_tri, NB);
      if (PREF && k > 0) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k - 1, 0), w, lane, up_tri, NB);
      acc_to_lds(acc, Vt, T, nullptr, w, cb0, lane);
      __syncthreads();
      // x_win = P^T [top ; carry]: rows that leave the window are emitted,
      // the others form the next carry in T1
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int64_t rows[RF];
        int cols[RF];
        cx<R> vals[RF];
        bool valid[RF];
#pragma unroll
        for (int q = 0; q < RF; ++q) {
          const int e = t + (h * RF + q) * NTHR;
          const int i = e / T, col = e % T;
          const cx<R> v = i < NB ? Vt[i * T + col] : Cb[(i - NB) * T + col];
          const int d = sp[i];
          valid[q] = d >= NB;
          rows[q] = (int64_t)k * NB + d;
          cols[q] = col;
          vals[q] = v;
          if (d < NB) T1[d * T + col] = v;
        }
        emit_batch(rows, cols, vals, valid);
      }
      __syncthreads();
      cx<R>* tmp = Cb;
      Cb = T1;
      T1 = tmp;
      if (k > 0) perm_store(pnext);
      __syncthreads();
    }
    {
      int64_t rows[RF];
      int cols[RF];
      cx<R> vals[RF];
      bool valid[RF];
#pragma unroll
      for (int q = 0; q < RF; ++q) {
        const int e = t + q * NTHR;
        valid[q] = true;
        rows[q] = e / T;
        cols[q] = e % T;
        vals[q] = Cb[e];
      }
      emit_batch(rows, cols, vals, valid);
    }
  }
}


template <typename R, int NB, int T, bool PREF, int NC, int OCC>
int launch_nb(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n, int njobs,
              const SolveJob* jobs_dev, hipStream_t st, const int32_t* gate) {
  const int K = (int)((n + NB - 1) / NB);
  size_t smem = solve_lds_bytes(NB, T, sizeof(cx<R>));
  (void)hipFuncSetAttribute((const void*)k_band_solve<R, NB, T, PREF, NC, OCC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
  for (int j0 = 0; j0 < njobs; j0 += 1 << 20) {
    int nj = njobs - j0 < (1 << 20) ? njobs - j0 : (1 << 20);
    int grid = 8 * ((nj + 7) / 8);
    k_band_solve<R, NB, T, PREF, NC, OCC><<<grid, NB * 4 * (T / (16 * NC)), smem, st>>>(
        mats, matsT, perm, n, K, jobs_dev + j0, nj, gate);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

template <typename R, int T, bool PREF, int NC, int OCC = 1>
int launch_t(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n, int nb,
             int njobs, const SolveJob* jobs_dev, hipStream_t st, const int32_t* gate) {
  switch (nb) {
    case 16: return launch_nb<R, 16, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 32: return launch_nb<R, 32, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 48: return launch_nb<R, 48, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 64: return launch_nb<R, 64, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 80: return launch_nb<R, 80, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 96: return launch_nb<R, 96, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 112: return launch_nb<R, 112, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 128: return launch_nb<R, 128, T, PREF, NC, OCC>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    default: return FB_ERR_INTERNAL;
  }
}

// every (tile width, prefetch, tiles per wave, register cap) variant of one precision
template <typename R>
int launch_variant(int variant, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                   int64_t n, int nb, int njobs, const SolveJob* jobs_dev, hipStream_t st,
                   const int32_t* gate) {
  switch (variant) {
    case 0: return launch_t<R, 16, false, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 1: return launch_t<R, 16, true, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 2: return launch_t<R, 32, false, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 3: return launch_t<R, 32, true, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 4: return launch_t<R, 32, false, 2>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 5: return launch_t<R, 32, true, 2>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 6: return launch_t<R, 16, false, 1, 3>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 7: return launch_t<R, 16, true, 1, 3>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    default: return FB_ERR_INTERNAL;
  }
}

}  // namespace fb
