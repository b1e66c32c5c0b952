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

// ---------------------------------------------------------------- chunk streaming
// The streamed form of a step's two block products: chunk ch is columns
// 16 ch .. 16 ch + 15 of op(A) for the wave's 16 rows (four complex values
// per lane), loaded RD chunks ahead of the MFMAs that use it, across the two
// products and into the next step (the carry), so that only RD + 1 chunks
// live in registers instead of whole fragments.  TR: element (i, k) of op(A)
// at A[i NB + k] (a conjugate transpose read from the block itself), else at
// A[k NB + i].
template <typename R>
struct Ck {
  cx<R> a[4];
};

template <typename R, int NB, bool TR>
__device__ __forceinline__ void ck_load(Ck<R>& c, const cx<R>* A, int w, int lane, int ch) {
  const int i = 16 * w + (lane & 15), kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = 16 * ch + 4 * q + kq;
    c.a[q] = TR ? A[(size_t)i * NB + k] : A[(size_t)k * NB + i];
  }
}

template <typename R, bool CONJT, bool NEG>
__device__ __forceinline__ void ck_mma(Acc<R, 1>& acc, const Ck<R>& c, const cx<R>* Bl, int ldb,
                                       const int* rmap, int cb0, int lane, int ch) {
  const int kq = lane >> 4, j = lane & 15;
  cx<R> bv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = 16 * ch + 4 * q + kq;
    const int br = rmap ? rmap[k] : k;
    bv[q] = Bl[(size_t)br * ldb + cb0 + j];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    R ar = c.a[q].x, ai = CONJT ? -c.a[q].y : c.a[q].y;
    if (NEG) {
      ar = -ar;
      ai = -ai;
    }
    acc.p1[0] = MF<R>::mma(ar, bv[q].x, acc.p1[0]);
    acc.p2[0] = MF<R>::mma(ai, bv[q].y, acc.p2[0]);
    acc.p3[0] = MF<R>::mma(ar + ai, bv[q].x + bv[q].y, acc.p3[0]);
  }
}

// acc += op(A0) B0 (NEG0: -=), mid(), acc += op(A1) B1 (NEG1: -=), both over
// all NB columns; carry holds the first RD chunks of A0 on entry and, when
// more, of Anext (the next step's A0) on exit (RD <= NB / 16).
template <typename R, int NB, bool TR, bool CONJT, bool NEG0, bool NEG1, int RD, class Mid>
__device__ __forceinline__ void stream_step(Acc<R, 1>& acc, Ck<R> (&carry)[RD], const cx<R>* A0,
                                            const cx<R>* A1, const cx<R>* Anext, bool more,
                                            const cx<R>* B0, const cx<R>* B1, const int* rm0,
                                            const int* rm1, int ldb, int cb0, int w, int lane,
                                            Mid mid) {
  constexpr int NCH = NB / 16, L = 2 * NCH;
  static_assert(RD >= 1 && RD <= NCH, "the carry holds chunks of the first product only");
  Ck<R> buf[L + RD];
#pragma unroll
  for (int i = 0; i < RD; ++i) buf[i] = carry[i];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int ip = i + RD;
    if (ip < L)
      ck_load<R, NB, TR>(buf[ip], ip < NCH ? A0 : A1, w, lane, ip % NCH);
    else if (more)
      ck_load<R, NB, TR>(buf[ip], Anext, w, lane, ip - L);
    if (i == NCH) mid();
    if (i < NCH)
      ck_mma<R, CONJT, NEG0>(acc, buf[i], B0, ldb, rm0, cb0, lane, i);
    else
      ck_mma<R, CONJT, NEG1>(acc, buf[i], B1, ldb, rm1, cb0, lane, i - NCH);
  }
#pragma unroll
  for (int i = 0; i < RD; ++i) carry[i] = buf[L + i];
}

// ---------------------------------------------------------------- MFMA block solve
// One workgroup per job with one wave per 16 x (16 NC) output tile of a block
// product ((NB/16) x (T/(16 NC)) waves; a wave with NC > 1 reuses each factor
// fragment for NC column tiles).  LDS holds 3 slots of NB x T (rows padded to
// T + 1 elements) and the block's permutation with its inverse.  Every tile
// that enters or leaves global memory goes through an LDS slot with thread
// e on row e % NB, column e / NB, so that a wave reads or writes whole column
// runs of 64 rows.  OCC > 1 asks the compiler to fit the registers of OCC
// waves per SIMD.
template <typename R, int NB, int T, bool PREF, int NC, int OCC, bool STR = false>
__global__ void __launch_bounds__(NB * 4 * (T / (16 * NC)), OCC)
k_band_solve(const cx<R>* __restrict__ mats, const cx<R>* __restrict__ matsT,
             const int16_t* __restrict__ permg, int64_t n, int K,
             const SolveJob* __restrict__ jobs, int njobs, const int32_t* __restrict__ gate) {
  // complex64 H solves read the transposed copy of the factor blocks
  constexpr bool TS = sizeof(R) == 4;
  constexpr int LDT = T + 1;    // LDS row of a slot
  constexpr int SL = NB * LDT;  // one slot
  extern __shared__ __align__(16) char lds_raw[];
  int* sp = reinterpret_cast<int*>(lds_raw);  // permutation, 2 NB entries
  int* si = sp + 2 * NB;                      // its inverse
  cx<R>* S = reinterpret_cast<cx<R>*>(lds_raw + ((4 * NB * sizeof(int) + 15) & ~15));
  const int job = remap_job(blockIdx.x, njobs);
  if (job >= njobs) return;
  const SolveJob jb = jobs[job];
  if (gate && !gate[jb.grp]) return;  // a correction its group no longer needs
  const int t = threadIdx.x, lane = t & 63;
  constexpr int NRW = NB / 16;
  // row block and column base of this wave (wave-uniform: scalar registers)
  const int w = __builtin_amdgcn_readfirstlane((t >> 6) % NRW);
  const int cb0 = __builtin_amdgcn_readfirstlane(16 * NC * ((t >> 6) / NRW));
  constexpr int NTHR = NB * 4 * (T / (16 * NC));
  constexpr int RF = NB * T / NTHR;  // tile elements per thread
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
  // tile element q of this thread: row e % NB, column e / NB
  auto erow = [&](int q) { return (t + q * NTHR) % NB; };
  auto ecol = [&](int q) { return (t + q * NTHR) / NB; };
  struct TileC {
    c128 v[RF];
  };
  struct TileR {
    cx<R> v[RF];
  };
  // global rows row0 .. row0 + NB - 1 of a tile into registers, then LDS
  auto tile_issue = [&](auto& f, auto base, int64_t ld, int64_t row0) {
#pragma unroll
    for (int q = 0; q < RF; ++q) f.v[q] = gld(gaddr(base, ld, row0 + erow(q), ecol(q)));
  };
  auto tile_store = [&](const auto& f, cx<R>* dst, int64_t row0) {
#pragma unroll
    for (int q = 0; q < RF; ++q)
      dst[erow(q) * LDT + ecol(q)] = conv(f.v[q], okf(row0 + erow(q), ecol(q)));
  };
  // values v[q] of rows row0 + erow(q) into the output (added to it for a
  // correction): all loads of the old values first, then the stores
  auto emit_vals = [&](const cx<R>* v, int64_t row0) {
    c128 old[RF];
    if (jb.add) {
#pragma unroll
      for (int q = 0; q < RF; ++q) old[q] = gld(gaddr(out, jb.ldout, row0 + erow(q), ecol(q)));
    }
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      const int64_t row = row0 + erow(q);
      if (!okf(row, ecol(q))) continue;
      c128 x = mk((double)v[q].x, (double)v[q].y);
      if (jb.add) x = old[q] + x;
      gst(out + (int64_t)ecol(q) * jb.ldout + row, x);
    }
  };
  auto emit_tile = [&](const cx<R>* src, int64_t row0) {
    cx<R> v[RF];
#pragma unroll
    for (int q = 0; q < RF; ++q) v[q] = src[erow(q) * LDT + ecol(q)];
    emit_vals(v, row0);
  };
  auto put_mid = [&](const cx<R>* src, int64_t row0) {
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      const int64_t row = row0 + erow(q);
      if (okf(row, ecol(q)))
        gst(mid + (int64_t)ecol(q) * jb.ldmid + row, src[erow(q) * LDT + ecol(q)]);
    }
  };
  auto zero_slots = [&](cx<R>* dst, int nslot) {
    for (int e = t; e < nslot * SL; e += NTHR) dst[e] = mk<R>(0, 0);
  };
  // the permutation of block k and its inverse
  auto perm_put = [&](int e, int v) {
    sp[e] = v;
    if ((unsigned)v < (unsigned)(2 * NB)) si[v] = e;
  };
  auto load_perm = [&](int k) {
    for (int e = t; e < 2 * NB; e += NTHR) perm_put(e, gld(P + (size_t)k * 2 * NB + e));
  };
  // fetched early into registers, stored later
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
      if (e < 2 * NB) perm_put(e, pp.v[q]);
    }
  };
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
  PreT<cx<R>, NC> pvm;  // intermediates (N backward)
  PreT<c128, NC> pvi;   // right-hand sides (H forward)

  if constexpr (STR) {
    static_assert(NC == 1, "streamed products take one 16-column tile per wave");
    // chunks in flight: the carry into the next step holds chunks of its
    // first product only, so at most that product's NB / 16 chunks
    constexpr int RD = NB >= 32 ? 2 : 1;
    Ck<R> carry[RD];
    auto none = [] {};
    if (jb.dir == 0) {
      // ------------------------------------------------------- N forward
      cx<R>* W = S;
      cx<R>* Yt = S + 2 * SL;
      {
        TileC f0, f1;
        tile_issue(f0, in, jb.ldin, 0);
        tile_issue(f1, in, jb.ldin, NB);
        tile_store(f0, W, 0);
        tile_store(f1, W + SL, NB);
      }
      TileC fr;
      load_perm(0);
#pragma unroll
      for (int i = 0; i < RD; ++i) ck_load<R, NB, false>(carry[i], blk(0, 0), w, lane, i);
      __syncthreads();
      for (int k = 0; k < K; ++k) {
        PermPre pnext;
        acc.zero();
        const bool more = k + 1 < K;
        stream_step<R, NB, false, false, false, true, RD>(
            acc, carry, blk(k, 0), blk(k, 1), blk(more ? k + 1 : k, 0), more, W, W, sp, sp, LDT,
            cb0, w, lane, [&] {
              acc_to_lds(acc, Yt, LDT, nullptr, w, cb0, lane);
              tile_issue(fr, in, jb.ldin, (int64_t)(k + 2) * NB);
              if (k + 1 < K) perm_issue(pnext, k + 1);
              acc_from_lds(acc, W, LDT, sp + NB, w, cb0, lane);
            });
        __syncthreads();
        acc_to_lds(acc, W, LDT, nullptr, w, cb0, lane);
        tile_store(fr, W + SL, (int64_t)(k + 2) * NB);
        put_mid(Yt, (int64_t)k * NB);
        if (k + 1 < K) perm_store(pnext);
        __syncthreads();
      }
      // ------------------------------------------------------- N backward
      // blocks beyond the last (G1(K-1), G2(K-2), G2(K-1)) are zero, as are
      // the x slots beyond x_{K-1}: every step runs both products
      cx<R>* X1 = S;
      cx<R>* X2 = S + SL;
      cx<R>* V = S + 2 * SL;
      zero_slots(S, 2);
      pre_load(pvm, mid, jb.ldmid, K - 1);
#pragma unroll
      for (int i = 0; i < RD; ++i) ck_load<R, NB, false>(carry[i], blk(K - 1, 3), w, lane, i);
      __syncthreads();
      for (int k = K - 1; k >= 0; --k) {
        pre_to_acc(acc, pvm);
        const bool more = k > 0;
        stream_step<R, NB, false, false, true, true, RD>(
            acc, carry, blk(k, 3), blk(k, 4), blk(more ? k - 1 : k, 3), more, X1, X2, nullptr,
            nullptr, LDT, cb0, w, lane, none);
        acc_to_lds(acc, V, LDT, nullptr, w, cb0, lane);
        if (k > 0) pre_load(pvm, mid, jb.ldmid, k - 1);
        if (k + 1 < K) emit_tile(X1, (int64_t)(k + 1) * NB);
        __syncthreads();
        cx<R>* tmp = X2;
        X2 = X1;
        X1 = V;
        V = tmp;
      }
      emit_tile(X1, 0);
    } else {
      // ------------------------------------------------------- H forward
      // G1(k-1)^H and G2(k-2)^H meet zero slots before the first steps
      // (block 0 stands in for the missing ones)
      constexpr bool TRH = !TS;
      cx<R>* W1 = S;
      cx<R>* W2 = S + SL;
      cx<R>* V = S + 2 * SL;
      zero_slots(S, 2);
      pre_load(pvi, in, jb.ldin, 0);
#pragma unroll
      for (int i = 0; i < RD; ++i) ck_load<R, NB, TRH>(carry[i], blkh(0, 3), w, lane, i);
      __syncthreads();
      for (int k = 0; k < K; ++k) {
        pre_to_acc(acc, pvi);
        const bool more = k + 1 < K;
        stream_step<R, NB, TRH, true, true, true, RD>(
            acc, carry, blkh(k >= 1 ? k - 1 : 0, 3), blkh(k >= 2 ? k - 2 : 0, 4), blkh(k, 3), more,
            W1, W2, nullptr, nullptr, LDT, cb0, w, lane, none);
        acc_to_lds(acc, V, LDT, nullptr, w, cb0, lane);
        if (k >= 1) put_mid(W1, (int64_t)(k - 1) * NB);
        if (k + 1 < K) pre_load(pvi, in, jb.ldin, k + 1);
        __syncthreads();
        cx<R>* tmp = W2;
        W2 = W1;
        W1 = V;
        V = tmp;
      }
      put_mid(W1, (int64_t)(K - 1) * NB);
      __syncthreads();
      // ------------------------------------------------------- H backward
      cx<R>* Cb = S;
      cx<R>* Wk = S + SL;
      cx<R>* Vt = S + 2 * SL;
      zero_slots(Cb, 1);
      {
        TileR f0;
        tile_issue(f0, mid, jb.ldmid, (int64_t)(K - 1) * NB);
        tile_store(f0, Wk, (int64_t)(K - 1) * NB);
      }
      load_perm(K - 1);
#pragma unroll
      for (int i = 0; i < RD; ++i) ck_load<R, NB, TRH>(carry[i], blkh(K - 1, 0), w, lane, i);
      __syncthreads();
      for (int k = K - 1; k >= 0; --k) {
        acc.zero();
        const bool more = k > 0;
        stream_step<R, NB, TRH, true, false, true, RD>(
            acc, carry, blkh(k, 0), blkh(k, 1), blkh(more ? k - 1 : k, 0), more, Wk, Cb, nullptr,
            nullptr, LDT, cb0, w, lane, none);
        TileR fw;
        PermPre pnext;
        if (k > 0) {
          tile_issue(fw, mid, jb.ldmid, (int64_t)(k - 1) * NB);
          perm_issue(pnext, k - 1);
        }
        acc_to_lds(acc, Vt, LDT, nullptr, w, cb0, lane);
        __syncthreads();
        {
          cx<R> cv[RF], lv[RF];
#pragma unroll
          for (int q = 0; q < RF; ++q) {
            const int r = erow(q), col = ecol(q);
            const int ic = si[r], il = si[NB + r];
            cv[q] = ic < NB ? Vt[ic * LDT + col] : Cb[(ic - NB) * LDT + col];
            lv[q] = il < NB ? Vt[il * LDT + col] : Cb[(il - NB) * LDT + col];
          }
#pragma unroll
          for (int q = 0; q < RF; ++q) Wk[erow(q) * LDT + ecol(q)] = cv[q];
          emit_vals(lv, (int64_t)k * NB + NB);
        }
        __syncthreads();
        if (k > 0) {
          tile_store(fw, Cb, (int64_t)(k - 1) * NB);
          perm_store(pnext);
        }
        cx<R>* tmp = Cb;
        Cb = Wk;
        Wk = tmp;
        __syncthreads();
      }
      emit_tile(Cb, 0);
    }
  } else {
    if (jb.dir == 0) {
      // ---------------------------------------------------------- N forward
      // v_k = Q z_top and the next window top z_bot - M z_top are both
      // products of z_top = rows sp[0, NB) of the window
      cx<R>* W = S;           // window: rows 0 .. 2 NB - 1 (two slots)
      cx<R>* Yt = S + 2 * SL; // v_k on its way to the intermediate
      {
        TileC f0, f1;
        tile_issue(f0, in, jb.ldin, 0);
        tile_issue(f1, in, jb.ldin, NB);
        tile_store(f0, W, 0);
        tile_store(f1, W + SL, NB);
      }
      TileC fr;
      load_perm(0);
      if (PREF) frag_load<R, NB, false>(fa, blk(0, 0), w, lane, 0, NB);
      __syncthreads();
      for (int k = 0; k < K; ++k) {
        if (PREF) frag_load<R, NB, false>(fb, blk(k, 1), w, lane, 0, NB);
        if (!PREF) frag_load<R, NB, false>(fa, blk(k, 0), w, lane, 0, NB);
        acc.zero();
        frag_mma<R, NB, NC, false, false>(acc, fa, W, LDT, sp, cb0, lane, 0, NB);
        acc_to_lds(acc, Yt, LDT, nullptr, w, cb0, lane);
        tile_issue(fr, in, jb.ldin, (int64_t)(k + 2) * NB);  // consumed after the product
        PermPre pnext;
        if (k + 1 < K) perm_issue(pnext, k + 1);
        if (PREF && k + 1 < K) frag_load<R, NB, false>(fa, blk(k + 1, 0), w, lane, 0, NB);
        if (!PREF) frag_load<R, NB, false>(fb, blk(k, 1), w, lane, 0, NB);
        acc_from_lds(acc, W, LDT, sp + NB, w, cb0, lane);
        frag_mma<R, NB, NC, false, true>(acc, fb, W, LDT, sp, cb0, lane, 0, NB);
        __syncthreads();
        acc_to_lds(acc, W, LDT, nullptr, w, cb0, lane);
        tile_store(fr, W + SL, (int64_t)(k + 2) * NB);
        put_mid(Yt, (int64_t)k * NB);
        if (k + 1 < K) perm_store(pnext);
        __syncthreads();
      }
      // ---------------------------------------------------------- N backward
      // x_k = v_k - G1 x_{k+1} - G2 x_{k+2}, one set of products per step;
      // x_{k+1} leaves for the output while step k runs
      cx<R>* X1 = S;
      cx<R>* X2 = S + SL;
      cx<R>* V = S + 2 * SL;
      zero_slots(S, 2);
      // fa = G1(k), fb = G2(k), pv = v_k: prefetched (the last step uses
      // neither block)
      pre_load(pvm, mid, jb.ldmid, K - 1);
      __syncthreads();
      for (int k = K - 1; k >= 0; --k) {
        if (!PREF && k + 1 < K) frag_load<R, NB, false>(fa, blk(k, 3), w, lane, 0, NB);
        if (!PREF && k + 2 < K) frag_load<R, NB, false>(fb, blk(k, 4), w, lane, 0, NB);
        pre_to_acc(acc, pvm);
        if (k + 1 < K) frag_mma<R, NB, NC, false, true>(acc, fa, X1, LDT, nullptr, cb0, lane, 0, NB);
        if (k + 2 < K) frag_mma<R, NB, NC, false, true>(acc, fb, X2, LDT, nullptr, cb0, lane, 0, NB);
        acc_to_lds(acc, V, LDT, nullptr, w, cb0, lane);
        if (k > 0) {
          if (PREF) frag_load<R, NB, false>(fa, blk(k - 1, 3), w, lane, 0, NB);
          if (PREF && k + 1 < K) frag_load<R, NB, false>(fb, blk(k - 1, 4), w, lane, 0, NB);
          pre_load(pvm, mid, jb.ldmid, k - 1);
        }
        if (k + 1 < K) emit_tile(X1, (int64_t)(k + 1) * NB);
        __syncthreads();
        cx<R>* tmp = X2;
        X2 = X1;
        X1 = V;
        V = tmp;
      }
      emit_tile(X1, 0);
    } else {
      // ---------------------------------------------------------- H forward (U^H)
      // u_k = y_k - G1(k-1)^H u_{k-1} - G2(k-2)^H u_{k-2}, one set of products
      // per step; u_{k-1} leaves for the intermediate while step k runs
      cx<R>* W1 = S;
      cx<R>* W2 = S + SL;
      cx<R>* V = S + 2 * SL;
      zero_slots(S, 2);
      // fa = G1(k-1)^H, fb = G2(k-2)^H, pv = y_k: prefetched
      pre_load(pvi, in, jb.ldin, 0);
      __syncthreads();
      for (int k = 0; k < K; ++k) {
        if (!PREF && k >= 1) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k - 1, 3), w, lane, 0, NB);
        if (!PREF && k >= 2) frag_load<R, NB, true, const cx<R>*, TS>(fb, blkh(k - 2, 4), w, lane, 0, NB);
        pre_to_acc(acc, pvi);
        if (k >= 1) frag_mma<R, NB, NC, true, true>(acc, fa, W1, LDT, nullptr, cb0, lane, 0, NB);
        if (k >= 2) frag_mma<R, NB, NC, true, true>(acc, fb, W2, LDT, nullptr, cb0, lane, 0, NB);
        acc_to_lds(acc, V, LDT, nullptr, w, cb0, lane);
        if (k + 1 < K) {
          if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k, 3), w, lane, 0, NB);
          if (PREF && k >= 1) frag_load<R, NB, true, const cx<R>*, TS>(fb, blkh(k - 1, 4), w, lane, 0, NB);
          pre_load(pvi, in, jb.ldin, k + 1);
        }
        if (k >= 1) put_mid(W1, (int64_t)(k - 1) * NB);
        __syncthreads();
        cx<R>* tmp = W2;
        W2 = W1;
        W1 = V;
        V = tmp;
      }
      put_mid(W1, (int64_t)(K - 1) * NB);
      __syncthreads();
      // ---------------------------------------------------------- H backward (L^H)
      // top = Q^H u_k - M^H carry from u_k and the carry in LDS; then
      // x_win = P^T [top ; carry], taken row by row through the inverse
      // permutation: window row si[d] lands on row d, rows d >= NB leave for the
      // output and rows d < NB form the next carry in the slot w_k held, and
      // w_{k-1} goes to the slot of the old carry.
      cx<R>* Cb = S;           // carry: window bottom
      cx<R>* Wk = S + SL;      // w_k, then the next carry
      cx<R>* Vt = S + 2 * SL;  // top of the window after the step
      zero_slots(Cb, 1);
      {
        TileR f0;
        tile_issue(f0, mid, jb.ldmid, (int64_t)(K - 1) * NB);
        tile_store(f0, Wk, (int64_t)(K - 1) * NB);
      }
      load_perm(K - 1);
      // fa = M^H, fc = Q^H
      if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(K - 1, 1), w, lane, 0, NB);
      if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(K - 1, 0), w, lane, 0, NB);
      __syncthreads();
      for (int k = K - 1; k >= 0; --k) {
        if (!PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k, 0), w, lane, 0, NB);
        acc.zero();
        frag_mma<R, NB, NC, true, false>(acc, fc, Wk, LDT, nullptr, cb0, lane, 0, NB);
        if (!PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k, 1), w, lane, 0, NB);
        frag_mma<R, NB, NC, true, true>(acc, fa, Cb, LDT, nullptr, cb0, lane, 0, NB);
        TileR fw;
        PermPre pnext;
        if (k > 0) {
          tile_issue(fw, mid, jb.ldmid, (int64_t)(k - 1) * NB);
          perm_issue(pnext, k - 1);
          if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fa, blkh(k - 1, 1), w, lane, 0, NB);
          if (PREF) frag_load<R, NB, true, const cx<R>*, TS>(fc, blkh(k - 1, 0), w, lane, 0, NB);
        }
        acc_to_lds(acc, Vt, LDT, nullptr, w, cb0, lane);
        __syncthreads();
        {
          cx<R> carry[RF], leave[RF];
  #pragma unroll
          for (int q = 0; q < RF; ++q) {
            const int r = erow(q), col = ecol(q);
            const int ic = si[r], il = si[NB + r];
            carry[q] = ic < NB ? Vt[ic * LDT + col] : Cb[(ic - NB) * LDT + col];
            leave[q] = il < NB ? Vt[il * LDT + col] : Cb[(il - NB) * LDT + col];
          }
  #pragma unroll
          for (int q = 0; q < RF; ++q) Wk[erow(q) * LDT + ecol(q)] = carry[q];
          emit_vals(leave, (int64_t)k * NB + NB);
        }
        __syncthreads();
        if (k > 0) {
          tile_store(fw, Cb, (int64_t)(k - 1) * NB);
          perm_store(pnext);
        }
        cx<R>* tmp = Cb;
        Cb = Wk;
        Wk = tmp;
        __syncthreads();
      }
      emit_tile(Cb, 0);
    }
  }
}


template <typename R, int NB, int T, bool PREF, int NC, int OCC, bool STR = false>
int launch_nb(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n, int njobs,
              const SolveJob* jobs_dev, hipStream_t st, const int32_t* gate) {
  const int K = (int)((n + NB - 1) / NB);
  size_t smem = solve_lds_bytes(NB, T, sizeof(cx<R>));
  (void)hipFuncSetAttribute((const void*)k_band_solve<R, NB, T, PREF, NC, OCC, STR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
  for (int j0 = 0; j0 < njobs; j0 += 1 << 20) {
    int nj = njobs - j0 < (1 << 20) ? njobs - j0 : (1 << 20);
    int grid = 8 * ((nj + 7) / 8);
    k_band_solve<R, NB, T, PREF, NC, OCC, STR><<<grid, NB * 4 * (T / (16 * NC)), smem, st>>>(
        mats, matsT, perm, n, K, jobs_dev + j0, nj, gate);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

template <typename R, int T, bool PREF, int NC, int OCC = 1, bool STR = false>
int launch_t(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n, int nb,
             int njobs, const SolveJob* jobs_dev, hipStream_t st, const int32_t* gate) {
  switch (nb) {
    case 16: return launch_nb<R, 16, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 32: return launch_nb<R, 32, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 48: return launch_nb<R, 48, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 64: return launch_nb<R, 64, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 80: return launch_nb<R, 80, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 96: return launch_nb<R, 96, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 112: return launch_nb<R, 112, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    case 128: return launch_nb<R, 128, T, PREF, NC, OCC, STR>(mats, matsT, perm, n, njobs, jobs_dev, st, gate);
    default: return FB_ERR_INTERNAL;
  }
}

// every (tile width, prefetch, tiles per wave, register cap) variant of one
// precision; in complex64, two tiles per wave ask for two waves per SIMD,
// which without the cap the compiler exceeds with accumulation registers
template <typename R>
int launch_variant(int variant, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                   int64_t n, int nb, int njobs, const SolveJob* jobs_dev, hipStream_t st,
                   const int32_t* gate) {
  // complex128 fragments are twice as wide: capped at two waves they spill
  constexpr int kOcc2 = sizeof(R) == 4 ? 2 : 1;
  // streamed products (8, 9): fragments no longer fill the registers
  constexpr int kOccS = 1;
  switch (variant) {
    case 0: return launch_t<R, 16, false, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 1: return launch_t<R, 16, true, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 2: return launch_t<R, 32, false, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 3: return launch_t<R, 32, true, 1>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 4: return launch_t<R, 32, false, 2, kOcc2>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 5: return launch_t<R, 32, true, 2, kOcc2>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 6: return launch_t<R, 16, false, 1, 3>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 7: return launch_t<R, 16, true, 1, 3>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 8: return launch_t<R, 16, false, 1, kOccS, true>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    case 9: return launch_t<R, 32, false, 1, kOccS, true>(mats, matsT, perm, n, nb, njobs, jobs_dev, st, gate);
    default: return FB_ERR_INTERNAL;
  }
}

}  // namespace fb
