// Band LU with partial pivoting of the shifted systems A = zI - B
// (one factorisation per integration node, Section 2.2, eq:feast_L2),
// producing the block form consumed by the block solves.
//
// One workgroup per system.  The active part of the elimination at step j is
// rows j..j+b and columns j..j+2b (U widens to bandwidth 2b under row
// interchanges); it lives in an MR x MC circular window (MR = b+2,
// MC = 2b+2) indexed by (physical row, column mod MC).  A logical row i
// maps to a physical row through phys[i mod MR] (held as the row's element
// offset, physical row times MC), so a row interchange is an O(1) swap of
// two table entries.  Row j+b+1 enters during step j into the
// physical row freed by row j-1, and its columns j+1 .. j+2b+1 are exactly
// the window's columns at step j+1.
//
// Output per block k of b columns (the window rows kb .. kb+2b-1):
//   perm  the net row permutation of the block's interchanges,
//   Lh11  unit lower multipliers of the top b rows (row-swapped as later
//         interchanges of the block move them, so that P A_panel = Lh U),
//   Lh21  multipliers of the bottom b rows,
//   U(k,k), U(k,k+1), U(k,k+2).
// A second kernel replaces Lh11 and U(k,k) by their inverses, a third Lh21
// by M = Lh21 Lh11^{-1}, and a fourth Lh11^{-1}, U(k,k+1) and U(k,k+2) by
// Q = U(k,k)^{-1} Lh11^{-1}, G1 = U(k,k)^{-1} U(k,k+1) and
// G2 = U(k,k)^{-1} U(k,k+2), so that each step of every solve sweep is one
// set of independent dense b x b products (see solve.hip).
//
// Within a block the multipliers are written to a per-system scratch under a
// storage row that follows each window row through the interchanges (an O(1)
// swap of two table entries), and gathered into row order once at the end of
// the block; the entering row of the next step is fetched from B while the
// current step runs.
#include "prof.h"
#include "solve_job.h"
#include "solve_kernel.h"

namespace fb {

static const int kLuThreads = 512;
static const size_t kLdsBudget = 160 * 1024;

template <typename R>
struct FactorOut {
  cx<R>* mats;     // nsys * K * 5 * b * b
  int16_t* perm;   // nsys * K * 2b
  int32_t* info;   // nsys
  cx<R>* lscr;     // nsys * 2 * 2b * b: multipliers of the current block by storage row
};

template <typename R, typename PB>
__device__ __forceinline__ cx<R> shifted_entry(PB Bd, int64_t n, int b, int64_t i, int64_t c,
                                               c128 z) {
  // A(i, c) of zI - B, padded with the identity beyond n
  if (i >= n || c >= n) return mk<R>(i == c ? (R)1 : (R)0, (R)0);
  int64_t d = i - c;
  c128 v;
  if (d >= 0) {
    if (d > b) return mk<R>(0, 0);
    c128 e = gld(Bd + d * n + c);
    v = mk(-e.x, -e.y);
  } else {
    if (-d > b) return mk<R>(0, 0);
    c128 e = gld(Bd + (-d) * n + i);
    v = mk(-e.x, e.y);  // -conj(B(c, i))
  }
  if (d == 0) {
    v.x += z.x;
    v.y = z.y;  // the diagonal of B is real
  }
  return mk<R>((R)v.x, (R)v.y);
}

// ---- wave-wide reductions of wave 0 for the pivot search, by DPP lane moves
// within rows of 16 lanes (xor 1, xor 2, half mirror, mirror) and reads of
// lanes 0, 16, 32 and 48; every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  return ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}
template <typename U, bool MAX>
__device__ __forceinline__ U wave_reduce(U v) {
  auto pick = [](U a, U b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
  if constexpr (sizeof(U) == 8) {
    v = pick(v, dpp64<0xB1>(v));   // quad_perm [1,0,3,2]
    v = pick(v, dpp64<0x4E>(v));   // quad_perm [2,3,0,1]
    v = pick(v, dpp64<0x141>(v));  // row_half_mirror
    v = pick(v, dpp64<0x140>(v));  // row_mirror
    return pick(pick(rdlane64(v, 0), rdlane64(v, 16)), pick(rdlane64(v, 32), rdlane64(v, 48)));
  } else {
    v = pick(v, dpp32<0xB1>(v));
    v = pick(v, dpp32<0x4E>(v));
    v = pick(v, dpp32<0x141>(v));
    v = pick(v, dpp32<0x140>(v));
    auto rd = [&](int l) { return (U)__builtin_amdgcn_readlane((int)v, l); };
    return pick(pick(rd(0), rd(16)), pick(rd(32), rd(48)));
  }
}
// bit pattern of a non-negative float or double: ordered as the value
__device__ __forceinline__ uint32_t ordered_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint64_t ordered_bits(double v) {
  return (uint64_t)__double_as_longlong(v);
}

// The elimination window: wholly in LDS, or split at element offset `split`
// (a whole number of physical rows) with the leading rows in LDS and the rest
// in the system's global scratch, so that only rows past the split add to
// the per-step global traffic and the cache footprint.  The split form's
// accesses are flat ones.
template <typename R, bool USE_LDS>
struct LuWindow {
  cx<R>* l;
  cx<R>* g;
  int split;
  __device__ __forceinline__ cx<R>& operator[](int e) const {
    if constexpr (USE_LDS)
      return l[e];
    else
      return *(e < split ? l + e : g + e);
  }
};

template <typename R, bool USE_LDS>
__global__ void __launch_bounds__(kLuThreads)
k_band_lu(const c128* __restrict__ Bd_, int64_t n, int b, int nb, int K,
          const c128* __restrict__ zs, FactorOut<R> out, cx<R>* __restrict__ gwin, int wsplit) {
  extern __shared__ __align__(16) char lds_raw[];
  const int MR = b + 2, MC = 2 * b + 2;
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t npad = (int64_t)K * nb;
  const c128 z = zs[s];

  // LDS: phys[MR] int, idx[2][2nb] int, piv info[4], lrow[2][2nb] int,
  // lvec[b+1] cx<R>, then the window
  int* phys = reinterpret_cast<int*>(lds_raw);
  int* idx = phys + MR;                   // two perm buffers (block parity)
  int* pivp = idx + 4 * nb;               // [0] = pivot row of this step
  int* lrow = pivp + 4;                   // two storage-row tables (block parity)
  cx<R>* lvec = reinterpret_cast<cx<R>*>(lds_raw + ((sizeof(int) * (MR + 8 * nb + 4) + 15) & ~15));
  // the window's memory is a compile-time choice, so that LDS accesses are
  // LDS instructions rather than flat ones where the whole window fits
  const LuWindow<R, USE_LDS> W{lvec + b + 1, USE_LDS ? nullptr : gwin + (size_t)s * MR * MC,
                               wsplit};
  const c128* Bd = Bd_;

  cx<R>* mats = out.mats + (size_t)s * K * 5 * nb * nb;
  int16_t* permg = out.perm + (size_t)s * K * 2 * nb;
  const size_t bb = (size_t)nb * nb;
  cx<R>* lscr = out.lscr + (size_t)s * 2 * 2 * bb;  // [parity][column][storage row]
  int32_t* info = out.info;

  // --- init: zero window, load rows 0..b, identity tables, zero block 0 scratch
  for (int e = t; e < MR * MC; e += blockDim.x) W[e] = mk<R>(0, 0);
  for (int e = t; e < MR; e += blockDim.x) phys[e] = e * MC;
  for (int e = t; e < 2 * nb; e += blockDim.x) {
    idx[e] = e;
    lrow[e] = e;
  }
  for (size_t e = t; e < 2 * bb; e += blockDim.x) gst(lscr + e, mk<R>(0, 0));
  if (t == 0) gst(info + s, 0);
  __syncthreads();
  {
    int64_t top = (int64_t)b < npad - 1 ? b : npad - 1;
    for (int e = t; e < (b + 1) * (2 * b + 1); e += blockDim.x) {
      int64_t i = e / (2 * b + 1), c = e % (2 * b + 1);
      if (i <= top && c < npad && c - i <= b && i - c <= b)
        W[i * MC + c] = shifted_entry<R>(Bd, n, b, i, c, z);
    }
  }
  __syncthreads();

  // entering row of step j (row j+b+1, columns j+1 .. j+2b+1): entry
  // e = t + q * kLuThreads of this thread, fetched one step ahead as the raw
  // complex128 element of B it comes from (B(i, c) at d = i - c = b - e >= 0,
  // B(c, i) above the diagonal), with a branch-free address, so that the
  // loads stay in flight until the row is stored a step later
  constexpr int ER = 2;  // 2b+1 <= 2 * kLuThreads for b <= 255
  auto fetch_row = [&](c128* raw, int64_t jf) {
    const int64_t inew = jf + b + 1;
#pragma unroll
    for (int q = 0; q < ER; ++q) {
      const int e = t + q * kLuThreads;
      const int64_t c = jf + 1 + e;
      const int d = b - e;
      const bool ok = e <= 2 * b && inew < n && c < n;
      const int64_t off = d >= 0 ? (int64_t)d * n + c : (int64_t)(-d) * n + inew;
      raw[q] = gld(Bd + (ok ? off : 0));
    }
  };
  // A(i, c) = z delta_ic - B(i, c) of the entering row from its raw element
  // (identity beyond n, zero beyond the padded order)
  auto row_entry = [&](c128 v, int64_t jf, int q) -> cx<R> {
    const int64_t inew = jf + b + 1;
    const int e = t + q * kLuThreads;
    const int64_t c = jf + 1 + e;
    const int d = b - e;
    if (e > 2 * b || inew >= npad || c >= npad) return mk<R>(0, 0);
    if (inew >= n || c >= n) return mk<R>(d == 0 ? (R)1 : (R)0, (R)0);
    if (d == 0) return mk<R>((R)(z.x - v.x), (R)z.y);  // the diagonal of B is real
    return d > 0 ? mk<R>((R)-v.x, (R)-v.y) : mk<R>((R)-v.x, (R)v.y);
  };

  // this thread's U-row entries e = t + q kLuThreads (e < 3 nb): block
  // 2 + e / nb, column e % nb, as an element offset within block row k
  constexpr int UR = 2;  // 3 nb <= 2 kLuThreads for nb <= 128
  size_t uoff[UR];
#pragma unroll
  for (int q = 0; q < UR; ++q) {
    const int e = t + q * kLuThreads;
    uoff[q] = (size_t)(2 + e / nb) * bb + (size_t)(e % nb) * nb;
  }

  // update mapping: 2b columns in flight, kLuThreads / 2b row groups
  const int ucols = 2 * b, ugrps = kLuThreads / ucols;
  const int ucol = t % ucols, ugrp = t / ucols;

  int first_zero = 0;
  // running slots: row j sits in slot jr = j mod MR, column j in jcs = j mod MC;
  // an offset below MR (MC) needs at most one wrap
  int jr = 0, jcs = 0, k = 0, jj = 0;
  auto rslot = [&](int off) { int v = jr + off; return v >= MR ? v - MR : v; };
  auto cslot = [&](int off) { int v = jcs + off; return v >= MC ? v - MC : v; };
  auto step = [&](int64_t j, const c128* cur, c128* nxt) {
    // Row j+b+1 enters (columns j+1 .. j+2b+1, fetched during the last step)
    // into the physical row that row j-1 left, and column j+2b+1 (the slot
    // column j-1 left) is zeroed in rows j .. j+b: after this step's
    // interchange rows j+1 .. j+b are among them, and the column is out of
    // their band.  Both slots are free since the end of the last step and
    // neither is read before the next barrier.  Storing them first, before
    // this step issues its own global loads and stores, means the wait for
    // the fetched row covers only memory operations a whole step old.
    if (j + b + 1 < npad) {
      const int pr = phys[rslot(b + 1)];
#pragma unroll
      for (int q = 0; q < ER; ++q) {
        const int e = t + q * kLuThreads;
        if (e <= 2 * b) W[pr + cslot(1 + e)] = row_entry(cur[q], j, q);
      }
    }
    {
      const int cs = cslot(2 * b + 1);
      for (int r = t; r <= b; r += blockDim.x) W[phys[rslot(r)] + cs] = mk<R>(0, 0);
    }
    if (j + 1 < npad) fetch_row(nxt, j + 1);
    const int par = k & 1;
    int* idxk = idx + par * 2 * nb;
    int* lrk = lrow + par * 2 * nb;
    cx<R>* scr = lscr + (size_t)par * 2 * bb;
    const int64_t last = (j + b < npad - 1) ? j + b : npad - 1;
    const int nr = (int)(last - j);               // rows below the pivot
    const int64_t cend = (j + 2 * b < npad - 1) ? j + 2 * b : npad - 1;
    const int nc = (int)(cend - j);               // columns right of the pivot
    const int jc = jcs;

    // ---- phase A (wave 0): pivot search, interchange, multipliers
    if (t < 64) {
      // largest |a|^2 of the column, ties to the lowest row: per lane over its
      // rows in increasing order, then the largest value over the wave and
      // the lowest row holding it
      R best = (R)0;
      int bi = 0x7fffffff;
      for (int r = t; r <= nr; r += 64) {
        cx<R> a = W[phys[rslot(r)] + jc];
        R v = cabs2(a);
        if (!(v >= (R)0)) v = (R)0;  // a NaN entry is never preferred
        if (bi == 0x7fffffff || v > best) {
          best = v;
          bi = r;
        }
      }
      {
        const auto mb = wave_reduce<decltype(ordered_bits(best)), true>(ordered_bits(best));
        const uint32_t cand =
            (bi != 0x7fffffff && ordered_bits(best) == mb) ? (uint32_t)bi : 0x7fffffffu;
        bi = (int)wave_reduce<uint32_t, false>(cand);
      }
      const int sj = jr, sp = rslot(bi);
      const int physj_old = phys[sj], physp_old = phys[sp];
      const int pw0 = jj + bi;
      cx<R> piv = W[physp_old + jc];
      cx<R> rp = cabs2(piv) > (R)0 ? cinv(piv) : mk<R>(0, 0);
      for (int r = t + 1; r <= nr; r += 64) {
        // after the interchange, window row jj + r holds the old row j when
        // r == bi; its storage row moves with it
        int pr = (r == bi) ? physj_old : phys[rslot(r)];
        int srow = (r == bi) ? lrk[jj] : lrk[jj + r];
        cx<R> l = W[pr + jc] * rp;
        lvec[r - 1] = l;
        gst(scr + (size_t)jj * 2 * nb + srow, l);
      }
      if (t == 0) {
        phys[sj] = physp_old;
        phys[sp] = physj_old;
        int a = idxk[jj];
        idxk[jj] = idxk[pw0];
        idxk[pw0] = a;
        a = lrk[jj];
        lrk[jj] = lrk[pw0];
        lrk[pw0] = a;
        pivp[0] = pw0;
        if (!(cabs2(piv) > (R)0) && first_zero == 0) first_zero = (int)(j + 1);
      }
    }
    __syncthreads();

    // ---- phase B (all): U row, update, entering row, block end
    const int prj = phys[jr];
    {
      // U row j: columns k nb .. k nb+3nb-1 of blocks U(k,k), U(k,k+1), U(k,k+2)
#pragma unroll
      for (int q = 0; q < UR; ++q) {
        const int e = t + q * kLuThreads;
        if (e >= 3 * nb) break;
        const int co = e - jj;  // column offset from j
        cx<R> v = mk<R>(0, 0);
        if (co >= 0 && co <= nc) v = W[prj + cslot(co)];
        gst(mats + (size_t)k * 5 * bb + uoff[q] + jj, v);
      }
      // rank-one update of rows j+1..last, columns j+1..cend: thread
      // (ucol, ugrp) keeps one column and walks every ugrps-th row
      if (ugrp < ugrps && ucol < nc) {
        const int cs = cslot(ucol + 1);
        const cx<R> u = W[prj + cs];
        // rows in batches of UB: all loads of a batch before its stores (the
        // rows are distinct physical rows, so nothing aliases)
        constexpr int UB = 8;
        for (int r0 = ugrp; r0 < nr; r0 += UB * ugrps) {
          int a[UB];
          cx<R> v[UB], l[UB];
          if (r0 + (UB - 1) * ugrps < nr) {
            // a whole batch in range (every batch but the last few steps'):
            // no per-row tests
#pragma unroll
            for (int q = 0; q < UB; ++q) a[q] = phys[rslot(r0 + q * ugrps + 1)] + cs;
#pragma unroll
            for (int q = 0; q < UB; ++q) {
              v[q] = W[a[q]];
              l[q] = lvec[r0 + q * ugrps];
            }
#pragma unroll
            for (int q = 0; q < UB; ++q) {
              v[q].x -= l[q].x * u.x - l[q].y * u.y;
              v[q].y -= l[q].x * u.y + l[q].y * u.x;
              W[a[q]] = v[q];
            }
            continue;
          }
#pragma unroll
          for (int q = 0; q < UB; ++q) {
            const int ro = r0 + q * ugrps;
            a[q] = ro < nr ? phys[rslot(ro + 1)] + cs : 0;
          }
#pragma unroll
          for (int q = 0; q < UB; ++q) {
            const int ro = r0 + q * ugrps;
            if (ro < nr) {
              v[q] = W[a[q]];
              l[q] = lvec[ro];
            }
          }
#pragma unroll
          for (int q = 0; q < UB; ++q) {
            const int ro = r0 + q * ugrps;
            if (ro < nr) {
              v[q].x -= l[q].x * u.x - l[q].y * u.y;
              v[q].y -= l[q].x * u.y + l[q].y * u.x;
              W[a[q]] = v[q];
            }
          }
        }
      }
      if (jj == nb - 1) {
        // block k complete: multipliers into row order (P A_panel = Lh U),
        // its permutation; fresh tables and scratch for block k+1
        // (batches of GB elements per thread: all loads of a batch, then
        // its stores)
        constexpr int GB = 8;
        const int nbb = 2 * (int)bb;  // 2 nb^2 <= 32768
        for (int e0 = t; e0 < nbb; e0 += GB * kLuThreads) {
          cx<R> v[GB];
#pragma unroll
          for (int q = 0; q < GB; ++q) {
            const int e = e0 + q * kLuThreads;
            const int ec = e < nbb ? e : 0;
            const int c = ec / (2 * nb), wr = ec - c * 2 * nb;
            v[q] = gld(scr + c * 2 * nb + lrk[wr]);
          }
#pragma unroll
          for (int q = 0; q < GB; ++q) {
            const int e = e0 + q * kLuThreads;
            if (e >= nbb) continue;
            const int c = e / (2 * nb), wr = e - c * 2 * nb;
            gst(mats + ((size_t)k * 5 + (wr < nb ? 0 : 1)) * bb + c * nb + (wr < nb ? wr : wr - nb),
                v[q]);
          }
        }
        cx<R>* scr1 = lscr + (size_t)(par ^ 1) * 2 * bb;
        for (size_t e = t; e < 2 * bb; e += blockDim.x) gst(scr1 + e, mk<R>(0, 0));
        for (int e = t; e < 2 * nb; e += blockDim.x) {
          gst(permg + (size_t)k * 2 * nb + e, (int16_t)idxk[e]);
          idx[(par ^ 1) * 2 * nb + e] = e;
          lrow[(par ^ 1) * 2 * nb + e] = e;
        }
      }
    }
    __syncthreads();
    jr = rslot(1);
    jcs = cslot(1);
    if (++jj == nb) {
      jj = 0;
      ++k;
    }
  };
  c128 ra[ER], rb[ER];
  fetch_row(ra, 0);
  for (int64_t j = 0; j < npad; j += 2) {
    step(j, ra, rb);
    if (j + 1 < npad) step(j + 1, rb, ra);
  }
  if (t == 0 && first_zero) gst(info + s, first_zero);
}

// In-place inverses of the unit lower Lh11 and the upper U(k,k) of every
// block by 16 x 16 tiles on MFMA: one workgroup per (system,
// block, which) and one wave per 16-column tile j of the inverse X, held in
// LDS (rows padded to 17 elements) by its rows that can be nonzero only:
// rows 16 j .. NB-1 of an L tile column, rows 0 .. 16 j + 15 of a U one,
// T (T + 1) / 2 tiles in all (T = NB / 16).  Each wave first inverts its diagonal
// tile by column recurrences on the already inverted part (16 lanes):
//   L = [1 0; l L22]:      L^{-1} column c below the diagonal = -L22^{-1} l
//   U = [U11 u; 0 ucc]:    U^{-1} column c above the diagonal = -U11^{-1} u / ucc
// then, after a barrier,
// runs the substitution down (L) or up (U) its tile column:
//   L: X(i,j) = -D(i)^{-1} sum_{k=j}^{i-1} L(i,k) X(k,j),   i = j+1 .. T-1
//   U: X(i,j) = -D(i)^{-1} sum_{k=i+1}^{j} U(i,k) X(k,j),   i = j-1 .. 0
// with D(i)^{-1} read from the diagonal tile of wave i's column; the sums
// are products of L or U tiles (fragments read from global memory) with the
// wave's own column (LDS), in Gauss form.  A wave hands values between its
// lanes through LDS under a wavefront fence.  All waves finish reading the
// block before the inverse is written over it.
template <typename R, int NB>
__global__ void __launch_bounds__(NB * 4)
k_block_invert_mfma(cx<R>* __restrict__ mats, int nblk) {
  constexpr int T = NB / 16;
  constexpr int LDT = 17;
  extern __shared__ __align__(16) char lds_raw[];
  cx<R>* Xs = reinterpret_cast<cx<R>*>(lds_raw);  // T (T + 1) / 2 tiles of 16 x LDT
  const int g = blockIdx.x;
  const int blk = g >> 1, which = g & 1;  // 0: Lh11 (slot 0), 1: U(k,k) (slot 2)
  if (blk >= nblk) return;
  cx<R>* M = mats + ((size_t)blk * 5 + (which ? 2 : 0)) * NB * NB;
  const int t = threadIdx.x, lane = t & 63;
  const int j = __builtin_amdgcn_readfirstlane(t >> 6);  // this wave's tile column
  // tile column i: X(r, c) at r LDT + c for its stored rows (16 i .. NB - 1 for
  // L, 0 .. 16 i + 15 for U); the tiles stored before it number
  // i T - i (i - 1) / 2 for L and i (i + 1) / 2 for U
  auto col = [&](int i) -> cx<R>* {
    const int before = which == 0 ? i * T - i * (i - 1) / 2 : i * (i + 1) / 2;
    const int r0 = which == 0 ? 16 * i : 0;
    return Xs + (size_t)(16 * before - r0) * LDT;
  };
  cx<R>* X = col(j);
  const int r0 = which == 0 ? 16 * j : 0;
  const int nrows = which == 0 ? NB - 16 * j : 16 * j + 16;
  auto wfence = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // the column tile's stored rows: zero, with the diagonal tile of M at rows 16 j ..
  for (int e = lane; e < nrows * 16; e += 64) {
    const int r = r0 + e % nrows, c = e / nrows;
    cx<R> v = mk<R>(0, 0);
    if (r >= 16 * j && r < 16 * j + 16) v = M[(size_t)(16 * j + c) * NB + r];
    X[r * LDT + c] = v;
  }
  wfence();
  cx<R>* D = X + 16 * j * LDT;  // D(r, c) at r LDT + c
  const int r = lane;
  if (which == 0) {
    // unit lower: column c below the diagonal = -Dinv22 l (trailing part done)
    for (int c = 14; c >= 0; --c) {
      cx<R> acc = mk<R>(0, 0);
      if (r > c && r < 16) {
        acc = D[r * LDT + c];
        for (int q = c + 1; q < r; ++q) cmac(acc, D[r * LDT + q], D[q * LDT + c]);
      }
      wfence();
      if (r > c && r < 16) D[r * LDT + c] = mk<R>(-acc.x, -acc.y);
      wfence();
    }
    if (r < 16) {
      D[r * LDT + r] = mk<R>((R)1, (R)0);
      for (int c = r + 1; c < 16; ++c) D[r * LDT + c] = mk<R>(0, 0);
    }
  } else {
    // upper: column c above the diagonal = -Dinv11 u / d_cc (leading part done)
    for (int c = 0; c < 16; ++c) {
      const cx<R> d = cinv(D[c * LDT + c]);
      cx<R> acc = mk<R>(0, 0);
      if (r < c) {
        for (int q = r; q < c; ++q) cmac(acc, D[r * LDT + q], D[q * LDT + c]);
        acc = acc * d;
      }
      wfence();
      if (r < c) D[r * LDT + c] = mk<R>(-acc.x, -acc.y);
      if (r == c) D[r * LDT + r] = d;
      wfence();
    }
    if (r < 16)
      for (int c = 0; c < r; ++c) D[r * LDT + c] = mk<R>(0, 0);
  }
  __syncthreads();
  // substitution along the tile column; fragments of the D(i)^{-1} tile:
  // register s holds D(i)^{-1}(lane % 16, 4 s + lane / 16)
  auto dinv_frag = [&](Frag<R, 16>& f, int i) {
    const cx<R>* Di = col(i) + 16 * i * LDT;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) f.a[s2] = Di[(lane & 15) * LDT + 4 * s2 + (lane >> 4)];
  };
  const int lo = which == 0 ? j + 1 : 0, hi = which == 0 ? T : j;
  for (int step = 0; step < hi - lo; ++step) {
    const int i = which == 0 ? lo + step : hi - 1 - step;
    const int k0 = which == 0 ? 16 * j : 16 * (i + 1);
    const int k1 = which == 0 ? 16 * i : 16 * (j + 1);
    Frag<R, NB> f;
    frag_load<R, NB, false>(f, (const cx<R>*)M, i, lane, k0, k1);
    Acc<R, 1> acc;
    acc.zero();
    frag_mma<R, NB, 1, false, false>(acc, f, X, LDT, nullptr, 0, lane, k0, k1);
    acc_to_lds(acc, X, LDT, nullptr, i, 0, lane);  // the sum, at rows 16 i ..
    wfence();
    Frag<R, 16> fd;
    dinv_frag(fd, i);
    Acc<R, 1> acc2;
    acc2.zero();
    frag_mma<R, 16, 1, false, true>(acc2, fd, X + 16 * i * LDT, LDT, nullptr, 0, lane, 0, 16);
    wfence();
    acc_to_lds(acc2, X, LDT, nullptr, i, 0, lane);
    wfence();
  }
  __syncthreads();  // every wave has read M
  for (int e = lane; e < NB * 16; e += 64) {
    const int rr = e % NB, c = e / NB;
    const bool stored = rr >= r0 && rr < r0 + nrows;
    gst(M + (size_t)(16 * j + c) * NB + rr, stored ? X[rr * LDT + c] : mk<R>(0, 0));
  }
}

template <typename R>
static size_t invert_mfma_lds_bytes(int nb) {
  const size_t t = (size_t)nb / 16;
  return sizeof(cx<R>) * (t * (t + 1) / 2) * 16 * 17;
}

template <typename R, int NB>
static int launch_invert_mfma_nb(cx<R>* mats, int nblk, hipStream_t st) {
  const size_t smem = invert_mfma_lds_bytes<R>(NB);
  if (smem > kLdsBudget) return FB_ERR_INTERNAL;
  (void)hipFuncSetAttribute((const void*)k_block_invert_mfma<R, NB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  k_block_invert_mfma<R, NB><<<2 * nblk, NB * 4, smem, st>>>(mats, nblk);
  FB_HIP(hipGetLastError());
  return 0;
}

// every block size up to 128 fits LDS in both precisions
template <typename R>
static int launch_invert_mfma(cx<R>* mats, int nb, int nblk, hipStream_t st) {
  if (invert_mfma_lds_bytes<R>(nb) > kLdsBudget) return FB_ERR_INTERNAL;
  int rc = 0;
  switch (nb) {
    case 16: rc = launch_invert_mfma_nb<R, 16>(mats, nblk, st); break;
    case 32: rc = launch_invert_mfma_nb<R, 32>(mats, nblk, st); break;
    case 48: rc = launch_invert_mfma_nb<R, 48>(mats, nblk, st); break;
    case 64: rc = launch_invert_mfma_nb<R, 64>(mats, nblk, st); break;
    case 80: rc = launch_invert_mfma_nb<R, 80>(mats, nblk, st); break;
    case 96: rc = launch_invert_mfma_nb<R, 96>(mats, nblk, st); break;
    case 112: rc = launch_invert_mfma_nb<R, 112>(mats, nblk, st); break;
    case 128: rc = launch_invert_mfma_nb<R, 128>(mats, nblk, st); break;
    default: return FB_ERR_INTERNAL;
  }
  return rc;
}

// M = Lh21 Lh11^{-1} in place of Lh21 (slot 1), one workgroup per block and
// one wave per 16 rows: a wave holds its rows of Lh21 as MFMA fragments and
// multiplies them by panels of PW columns of the lower triangular inverse
// staged in LDS (rows below the panel's first column only).  A wave reads and
// writes only its own rows of the slot.
template <typename R, int NB>
__global__ void __launch_bounds__(NB * 4)
k_form_m(cx<R>* __restrict__ mats, int nblk) {
  constexpr int PW = NB < 64 ? NB : 64;
  constexpr int NC = PW / 16;
  constexpr int LD = PW + 1;
  extern __shared__ __align__(16) char lds_raw[];
  cx<R>* Lp = reinterpret_cast<cx<R>*>(lds_raw);  // NB x LD: Lh11^{-1}(k, p0 + c) at k LD + c
  const int blk = blockIdx.x;
  if (blk >= nblk) return;
  const cx<R>* Li = mats + ((size_t)blk * 5 + 0) * NB * NB;
  cx<R>* L21 = mats + ((size_t)blk * 5 + 1) * NB * NB;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  Frag<R, NB> f;
  frag_load<R, NB, false>(f, L21, w, lane, 0, NB);
  for (int p0 = 0; p0 < NB; p0 += PW) {
    __syncthreads();
    // the last panel of a block that PW does not divide is partial: its
    // columns beyond the block are zeros and are not written
    for (int e = t; e < NB * PW; e += NB * 4) {
      const int k = e % NB, c = e / NB;
      Lp[k * LD + c] = p0 + c < NB ? Li[(size_t)(p0 + c) * NB + k] : mk<R>(0, 0);
    }
    __syncthreads();
    Acc<R, NC> acc;
    acc.zero();
    frag_mma<R, NB, NC, false, false>(acc, f, Lp, LD, nullptr, 0, lane, p0, NB);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + MF<R>::row(lane, r);
        const int col = p0 + 16 * c + (lane & 15);
        if (col < NB) gst(L21 + (size_t)col * NB + row, acc.get(c, r));
      }
  }
}

template <typename R, int NB>
static int launch_form_m_nb(cx<R>* mats, int nblk, hipStream_t st) {
  constexpr int PW = NB < 64 ? NB : 64;
  const size_t smem = sizeof(cx<R>) * (size_t)NB * (PW + 1);
  (void)hipFuncSetAttribute((const void*)k_form_m<R, NB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  k_form_m<R, NB><<<nblk, NB * 4, smem, st>>>(mats, nblk);
  FB_HIP(hipGetLastError());
  return 0;
}

template <typename R>
static int launch_form_m(cx<R>* mats, int nb, int nblk, hipStream_t st) {
  switch (nb) {
    case 16: return launch_form_m_nb<R, 16>(mats, nblk, st);
    case 32: return launch_form_m_nb<R, 32>(mats, nblk, st);
    case 48: return launch_form_m_nb<R, 48>(mats, nblk, st);
    case 64: return launch_form_m_nb<R, 64>(mats, nblk, st);
    case 80: return launch_form_m_nb<R, 80>(mats, nblk, st);
    case 96: return launch_form_m_nb<R, 96>(mats, nblk, st);
    case 112: return launch_form_m_nb<R, 112>(mats, nblk, st);
    case 128: return launch_form_m_nb<R, 128>(mats, nblk, st);
    default: return FB_ERR_INTERNAL;
  }
}

// The blocks that let every solve sweep take one product phase per block
// row, from the inverses (slot 2: U(k,k)^{-1}, slot 0: Lh11^{-1}) and U's
// off-diagonal blocks:
//   Q  = U(k,k)^{-1} Lh11^{-1}  in place of Lh11^{-1} (slot 0),
//   G1 = U(k,k)^{-1} U(k,k+1)   in place of U(k,k+1)  (slot 3),
//   G2 = U(k,k)^{-1} U(k,k+2)   in place of U(k,k+2)  (slot 4).
// One workgroup per block and one wave per 16 rows: a wave holds its rows of
// the upper triangular inverse as MFMA fragments and multiplies them by
// panels of PW columns of each right operand staged in LDS, with the
// triangles that vanish in exact arithmetic (below the diagonal of U(k,k)^{-1},
// above it in Lh11^{-1} and U(k,k+2)) taken as zeros.  A panel is staged
// before any wave overwrites its columns.  Runs after k_form_m, which reads
// Lh11^{-1}.
template <typename R, int NB>
__global__ void __launch_bounds__(NB * 4)
k_form_qg(cx<R>* __restrict__ mats, int nblk) {
  constexpr int PW = NB < 64 ? NB : 64;
  constexpr int NC = PW / 16;
  constexpr int LD = PW + 1;
  extern __shared__ __align__(16) char lds_raw[];
  cx<R>* Bp = reinterpret_cast<cx<R>*>(lds_raw);  // NB x LD: operand(k, p0 + c) at k LD + c
  const int blk = blockIdx.x;
  if (blk >= nblk) return;
  cx<R>* base = mats + (size_t)blk * 5 * NB * NB;
  const cx<R>* Ui = base + (size_t)2 * NB * NB;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  Frag<R, NB> f;
  frag_load<R, NB, false>(f, Ui, w, lane, 16 * w, NB);
  {
    // fragment s holds row 16 w + lane % 16, column 4 s + lane / 16
    const int i = 16 * w + (lane & 15);
#pragma unroll
    for (int s = 0; s < NB / 4; ++s)
      if (4 * s + (lane >> 4) < i) f.a[s] = mk<R>(0, 0);
  }
  for (int which = 0; which < 3; ++which) {
    cx<R>* O = base + (size_t)(which == 0 ? 0 : which + 2) * NB * NB;
    const bool lower = which != 1;  // Lh11^{-1} and U(k,k+2)
    for (int p0 = 0; p0 < NB; p0 += PW) {
      __syncthreads();
      for (int e = t; e < NB * PW; e += NB * 4) {
        const int k = e % NB, c = e / NB;
        // a partial last panel (PW does not divide NB): zeros beyond the block
        cx<R> v = p0 + c < NB ? O[(size_t)(p0 + c) * NB + k] : mk<R>(0, 0);
        if (lower && k < p0 + c) v = mk<R>(0, 0);
        Bp[k * LD + c] = v;
      }
      __syncthreads();
      Acc<R, NC> acc;
      acc.zero();
      frag_mma<R, NB, NC, false, false>(acc, f, Bp, LD, nullptr, 0, lane, 16 * w, NB);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * w + MF<R>::row(lane, r);
          const int col = p0 + 16 * c + (lane & 15);
          if (col < NB) gst(O + (size_t)col * NB + row, acc.get(c, r));
        }
    }
  }
}

template <typename R, int NB>
static int launch_form_qg_nb(cx<R>* mats, int nblk, hipStream_t st) {
  constexpr int PW = NB < 64 ? NB : 64;
  const size_t smem = sizeof(cx<R>) * (size_t)NB * (PW + 1);
  (void)hipFuncSetAttribute((const void*)k_form_qg<R, NB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  k_form_qg<R, NB><<<nblk, NB * 4, smem, st>>>(mats, nblk);
  FB_HIP(hipGetLastError());
  return 0;
}

template <typename R>
static int launch_form_qg(cx<R>* mats, int nb, int nblk, hipStream_t st) {
  switch (nb) {
    case 16: return launch_form_qg_nb<R, 16>(mats, nblk, st);
    case 32: return launch_form_qg_nb<R, 32>(mats, nblk, st);
    case 48: return launch_form_qg_nb<R, 48>(mats, nblk, st);
    case 64: return launch_form_qg_nb<R, 64>(mats, nblk, st);
    case 80: return launch_form_qg_nb<R, 80>(mats, nblk, st);
    case 96: return launch_form_qg_nb<R, 96>(mats, nblk, st);
    case 112: return launch_form_qg_nb<R, 112>(mats, nblk, st);
    case 128: return launch_form_qg_nb<R, 128>(mats, nblk, st);
    default: return FB_ERR_INTERNAL;
  }
}

template <typename R>
static size_t lu_lds_head_bytes(int b) {
  const int nb = block_size(b);
  size_t head = (sizeof(int) * (size_t)((b + 2) + 8 * nb + 4) + 15) & ~(size_t)15;
  return head + sizeof(cx<R>) * ((size_t)b + 1);
}
template <typename R>
static size_t lu_lds_bytes(int b) {
  return lu_lds_head_bytes<R>(b) + sizeof(cx<R>) * (size_t)(b + 2) * (2 * b + 2);
}

// whole window rows that fit in LDS beside the head when the window does not
template <typename R>
static int lu_lds_rows(int b) {
  const size_t row = sizeof(cx<R>) * (size_t)(2 * b + 2);
  const size_t head = lu_lds_head_bytes<R>(b);
  const size_t rows = head < kLdsBudget ? (kLdsBudget - head) / row : 0;
  return (int)std::min<size_t>(rows, (size_t)b + 2);
}

template <typename R>
size_t lu_window_scratch(int b, int nsys) {
  if (lu_lds_bytes<R>(b) <= kLdsBudget) return 0;
  return (size_t)nsys * (b + 2) * (2 * b + 2) * sizeof(cx<R>);
}

// Transposed copy of every nb x nb factor block (32 x 32 tiles through LDS),
// read by the conjugate-transposed solves so that a wave's factor fragment
// loads are contiguous along the block's rows.
template <typename R>
__global__ void __launch_bounds__(256)
k_transpose_blocks(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst, int nb) {
  __shared__ cx<R> tile[32][33];
  const size_t bb = (size_t)nb * nb;
  const cx<R>* S = src + (size_t)blockIdx.x * bb;
  cx<R>* D = dst + (size_t)blockIdx.x * bb;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int i0 = 0; i0 < nb; i0 += 32)
    for (int j0 = 0; j0 < nb; j0 += 32) {
      // tile of S at rows i0.., columns j0.. (element (i, j) at j * nb + i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + ty + 8 * q, i = i0 + tx;
        if (i < nb && j < nb) tile[ty + 8 * q][tx] = gld(S + (size_t)j * nb + i);
      }
      __syncthreads();
      // D(j, i) = S(i, j): D element (j, i) at i * nb + j
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + ty + 8 * q, j = j0 + tx;
        if (i < nb && j < nb) gst(D + (size_t)i * nb + j, tile[tx][ty + 8 * q]);
      }
      __syncthreads();
    }
}

template <typename R>
int launch_lu_impl(const Band& bd, int nsys, const c128* z_dev, cx<R>* mats, cx<R>* matsT,
                   int16_t* perm, int32_t* info, cx<R>* scratch, cx<R>* lscr, hipStream_t st) {
  const int b = bd.b;
  const int nb = block_size(b);
  const int K = (int)((bd.n + nb - 1) / nb);
  FactorOut<R> o{mats, perm, info, lscr};
  bool lds = lu_lds_bytes<R>(b) <= kLdsBudget;
  // split window: the leading physical rows that fit stay in LDS
  const int lrows = lds ? b + 2 : lu_lds_rows<R>(b);
  const int wsplit = lrows * (2 * b + 2);
  size_t smem = lds ? lu_lds_bytes<R>(b)
                    : lu_lds_head_bytes<R>(b) + sizeof(cx<R>) * (size_t)wsplit;
  if (smem > kLdsBudget) return FB_ERR_INTERNAL;
  (void)hipFuncSetAttribute((const void*)k_band_lu<R, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipFuncSetAttribute((const void*)k_band_lu<R, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  {
    ProfScope ps(FB_PROF_LU, st, 16.0 * (double)bd.n * b * b * nsys);
    if (lds)
      k_band_lu<R, true><<<nsys, kLuThreads, smem, st>>>(bd.Bd, bd.n, b, nb, K, z_dev, o, scratch,
                                                         wsplit);
    else
      k_band_lu<R, false><<<nsys, kLuThreads, smem, st>>>(bd.Bd, bd.n, b, nb, K, z_dev, o, scratch,
                                                          wsplit);
    FB_HIP(hipGetLastError());
  }
  int nblk = nsys * K;
  // inverses (2 nb^3 / 3 complex multiply-adds per block), M (nb^3 / 2) and
  // Q, G1, G2 (nb^3 / 3 + nb^3 / 2 + nb^3 / 3)
  ProfScope ps(FB_PROF_INVERT, st,
               8.0 * nblk * (double)nb * nb * nb * (2.0 / 3.0 + 0.5 + 7.0 / 6.0));
  FB_TRY(launch_invert_mfma<R>(mats, nb, nblk, st));
  FB_TRY(launch_form_m<R>(mats, nb, nblk, st));
  FB_TRY(launch_form_qg<R>(mats, nb, nblk, st));
  if (matsT) {
    k_transpose_blocks<R><<<5 * nblk, 256, 0, st>>>(mats, matsT, nb);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

template int launch_lu_impl<float>(const Band&, int, const c128*, c64*, c64*, int16_t*,
                                   int32_t*, c64*, c64*, hipStream_t);
template int launch_lu_impl<double>(const Band&, int, const c128*, c128*, c128*, int16_t*,
                                    int32_t*, c128*, c128*, hipStream_t);
template size_t lu_window_scratch<float>(int, int);
template size_t lu_window_scratch<double>(int, int);

}  // namespace fb
