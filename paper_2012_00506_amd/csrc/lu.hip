// Band LU with partial pivoting of the shifted systems A = zI - B
// (one factorisation per integration node, Section 2.2, eq:feast_L2),
// producing the block form consumed by the block solves.
//
// One workgroup per system.  The active part of the elimination at step j is
// rows j..j+b and columns j..j+2b (U widens to bandwidth 2b under row
// interchanges); it lives in an MR x MC circular window (MR = b+2,
// MC = 2b+2) indexed by (physical row, column mod MC).  A logical row i
// maps to a physical row through phys[i mod MR], so a row interchange is
// an O(1) swap of two table entries.  Row j+b+1 enters during step j into the
// physical row freed by row j-1, and its columns j+1 .. j+2b+1 are exactly
// the window's columns at step j+1.
//
// Output per block k of b columns (the window rows kb .. kb+2b-1):
//   perm  the net row permutation of the block's interchanges,
//   Lh11  unit lower multipliers of the top b rows (row-swapped as later
//         interchanges of the block move them, so that P A_panel = Lh U),
//   Lh21  multipliers of the bottom b rows,
//   U(k,k), U(k,k+1), U(k,k+2).
// A second kernel replaces Lh11 and U(k,k) by their inverses, so that the
// solves are chains of dense b x b products.
//
// Within a block the multipliers are written to a per-system scratch under a
// storage row that follows each window row through the interchanges (an O(1)
// swap of two table entries), and gathered into row order once at the end of
// the block; the entering row of the next step is fetched from B while the
// current step runs.
#include "solve_job.h"
#include "prof.h"

namespace fb {

static const int kLuThreads = 256;
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

template <typename R, bool USE_LDS>
__global__ void __launch_bounds__(kLuThreads)
k_band_lu(const c128* __restrict__ Bd_, int64_t n, int b, int nb, int K,
          const c128* __restrict__ zs, FactorOut<R> out, cx<R>* __restrict__ gwin) {
  extern __shared__ char lds_raw[];
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
  // LDS instructions rather than flat ones
  cx<R>* W = USE_LDS ? lvec + b + 1 : gwin + (size_t)s * MR * MC;
  const c128* Bd = Bd_;

  cx<R>* mats = out.mats + (size_t)s * K * 5 * nb * nb;
  int16_t* permg = out.perm + (size_t)s * K * 2 * nb;
  const size_t bb = (size_t)nb * nb;
  cx<R>* lscr = out.lscr + (size_t)s * 2 * 2 * bb;  // [parity][column][storage row]
  int32_t* info = out.info;

  // --- init: zero window, load rows 0..b, identity tables, zero block 0 scratch
  for (int e = t; e < MR * MC; e += blockDim.x) W[e] = mk<R>(0, 0);
  for (int e = t; e < MR; e += blockDim.x) phys[e] = e;
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
  // e = t + q * kLuThreads of this thread, fetched one step ahead
  constexpr int ER = 2;  // 2b+1 <= 2 * kLuThreads for b <= 255
  auto fetch_row = [&](cx<R>* dst, int64_t jf) {
    const int64_t inew = jf + b + 1;
#pragma unroll
    for (int q = 0; q < ER; ++q) {
      const int e = t + q * kLuThreads;
      cx<R> v = mk<R>(0, 0);
      if (e <= 2 * b && inew < npad) {
        const int64_t c = jf + 1 + e;
        if (c < npad) v = shifted_entry<R>(Bd, n, b, inew, c, z);
      }
      dst[q] = v;
    }
  };

  // update mapping: 2b columns in flight, kLuThreads / 2b row groups
  const int ucols = 2 * b, ugrps = kLuThreads / ucols;
  const int ucol = t % ucols, ugrp = t / ucols;

  int first_zero = 0;
  // running slots: row j sits in slot jr = j mod MR, column j in jcs = j mod MC;
  // an offset below MR (MC) needs at most one wrap
  int jr = 0, jcs = 0, k = 0, jj = 0;
  auto rslot = [&](int off) { int v = jr + off; return v >= MR ? v - MR : v; };
  auto cslot = [&](int off) { int v = jcs + off; return v >= MC ? v - MC : v; };
  auto step = [&](int64_t j, const cx<R>* cur, cx<R>* nxt) {
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
      R best = (R)-1;
      int bi = 0x7fffffff;
      for (int r = t; r <= nr; r += 64) {
        cx<R> a = W[(size_t)phys[rslot(r)] * MC + jc];
        R v = cabs2(a);
        if (v > best) {  // rows scanned in increasing order per lane
          best = v;
          bi = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        R ob = __shfl_xor(best, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      const int sj = jr, sp = rslot(bi);
      const int physj_old = phys[sj], physp_old = phys[sp];
      const int pw0 = jj + bi;
      cx<R> piv = W[(size_t)physp_old * MC + jc];
      cx<R> rp = cabs2(piv) > (R)0 ? cinv(piv) : mk<R>(0, 0);
      for (int r = t + 1; r <= nr; r += 64) {
        // after the interchange, window row jj + r holds the old row j when
        // r == bi; its storage row moves with it
        int pr = (r == bi) ? physj_old : phys[rslot(r)];
        int srow = (r == bi) ? lrk[jj] : lrk[jj + r];
        cx<R> l = W[(size_t)pr * MC + jc] * rp;
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
      for (int e = t; e < 3 * nb; e += blockDim.x) {
        int co = e - jj;  // column offset from j
        cx<R> v = mk<R>(0, 0);
        if (co >= 0 && co <= nc) v = W[(size_t)prj * MC + cslot(co)];
        int which = 2 + e / nb;
        gst(mats + ((size_t)k * 5 + which) * bb + (size_t)(e % nb) * nb + jj, v);
      }
      // rank-one update of rows j+1..last, columns j+1..cend: thread
      // (ucol, ugrp) keeps one column and walks every ugrps-th row
      if (ugrp < ugrps && ucol < nc) {
        const int cs = cslot(ucol + 1);
        const cx<R> u = W[(size_t)prj * MC + cs];
        // rows in batches of UB: all loads of a batch before its stores (the
        // rows are distinct physical rows, so nothing aliases)
        constexpr int UB = 8;
        for (int r0 = ugrp; r0 < nr; r0 += UB * ugrps) {
          size_t a[UB];
          cx<R> v[UB], l[UB];
#pragma unroll
          for (int q = 0; q < UB; ++q) {
            const int ro = r0 + q * ugrps;
            a[q] = ro < nr ? (size_t)phys[rslot(ro + 1)] * MC + cs : 0;
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
      // column j+2b+1 enters: zero it in rows j+1..j+b (out of their band)
      {
        int cs = cslot(2 * b + 1);
        for (int r = t; r < b; r += blockDim.x) W[(size_t)phys[rslot(r + 1)] * MC + cs] = mk<R>(0, 0);
      }
      // row j+b+1 enters (columns j+1 .. j+2b+1), fetched during the last step
      if (j + b + 1 < npad) {
        int pr = phys[rslot(b + 1)];
#pragma unroll
        for (int q = 0; q < ER; ++q) {
          const int e = t + q * kLuThreads;
          if (e <= 2 * b) W[(size_t)pr * MC + cslot(1 + e)] = cur[q];
        }
      }
      if (jj == nb - 1) {
        // block k complete: multipliers into row order (P A_panel = Lh U),
        // its permutation; fresh tables and scratch for block k+1
        for (size_t e = t; e < 2 * bb; e += blockDim.x) {
          const int c = (int)(e / (2 * nb)), wr = (int)(e % (2 * nb));
          cx<R> v = gld(scr + (size_t)c * 2 * nb + lrk[wr]);
          gst(mats + ((size_t)k * 5 + (wr < nb ? 0 : 1)) * bb + (size_t)c * nb + (wr < nb ? wr : wr - nb), v);
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
  cx<R> ra[ER], rb[ER];
  fetch_row(ra, 0);
  for (int64_t j = 0; j < npad; j += 2) {
    step(j, ra, rb);
    if (j + 1 < npad) step(j + 1, rb, ra);
  }
  if (t == 0 && first_zero) gst(info + s, first_zero);
}

// In-place inverses of the unit lower Lh11 and the upper U(k,k) of every
// block: one workgroup per (system, block, which).  Column recurrences on the
// already inverted part (trailing part for L, leading part for U):
//   L = [1 0; l L22]:      L^{-1} column j below the diagonal = -L22^{-1} l
//   U = [U11 u; 0 ujj]:    U^{-1} column j above the diagonal = -U11^{-1} u / ujj
// The matrix is staged in LDS when it fits, else worked on in place in global
// memory; only the column being replaced is copied aside.
template <typename R, bool USE_LDS>
__global__ void __launch_bounds__(256)
k_block_invert(cx<R>* __restrict__ mats, int b, int nblk) {
  extern __shared__ char lds_raw[];
  const int g = blockIdx.x;
  const int blk = g >> 1, which = g & 1;  // 0: Lh11 (slot 0), 1: U(k,k) (slot 2)
  if (blk >= nblk) return;
  cx<R>* M = mats + ((size_t)blk * 5 + (which ? 2 : 0)) * b * b;
  cx<R>* xv = reinterpret_cast<cx<R>*>(lds_raw);
  cx<R>* A = USE_LDS ? xv + b : M;
  const int t = threadIdx.x;
  const int bb = b * b;
  if (USE_LDS) {
    for (int e = t; e < bb; e += blockDim.x) A[e] = M[e];
    __syncthreads();
  }
  if (which == 0) {
    for (int j = b - 2; j >= 0; --j) {
      for (int i = j + 1 + t; i < b; i += blockDim.x) xv[i] = A[j * b + i];
      __syncthreads();
      for (int r = j + 1 + t; r < b; r += blockDim.x) {
        cx<R> acc = xv[r];  // unit diagonal of the inverted trailing block
        for (int q = j + 1; q < r; ++q) cmac(acc, A[q * b + r], xv[q]);
        A[j * b + r] = mk<R>(-acc.x, -acc.y);
      }
      __syncthreads();
    }
    for (int j = t; j < b; j += blockDim.x) A[j * b + j] = mk<R>((R)1, (R)0);
  } else {
    for (int j = 0; j < b; ++j) {
      for (int i = t; i <= j; i += blockDim.x) xv[i] = A[j * b + i];
      __syncthreads();
      cx<R> d = cinv(xv[j]);
      for (int r = t; r < j; r += blockDim.x) {
        cx<R> acc = mk<R>(0, 0);
        for (int q = r; q < j; ++q) cmac(acc, A[q * b + r], xv[q]);
        acc = acc * d;
        A[j * b + r] = mk<R>(-acc.x, -acc.y);
      }
      if (t == 0) A[j * b + j] = d;
      __syncthreads();
    }
  }
  __syncthreads();
  if (USE_LDS)
    for (int e = t; e < bb; e += blockDim.x) M[e] = A[e];
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

template <typename R>
size_t lu_window_scratch(int b, int nsys) {
  if (lu_lds_bytes<R>(b) <= kLdsBudget) return 0;
  return (size_t)nsys * (b + 2) * (2 * b + 2) * sizeof(cx<R>);
}

template <typename R>
int launch_lu_impl(const Band& bd, int nsys, const c128* z_dev, cx<R>* mats, int16_t* perm,
                   int32_t* info, cx<R>* scratch, cx<R>* lscr, hipStream_t st) {
  const int b = bd.b;
  const int nb = block_size(b);
  const int K = (int)((bd.n + nb - 1) / nb);
  FactorOut<R> o{mats, perm, info, lscr};
  bool lds = lu_lds_bytes<R>(b) <= kLdsBudget;
  size_t smem = lds ? lu_lds_bytes<R>(b) : lu_lds_head_bytes<R>(b);
  (void)hipFuncSetAttribute((const void*)k_band_lu<R, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  {
    ProfScope ps(FB_PROF_LU, st, 16.0 * (double)bd.n * b * b * nsys);
    if (lds)
      k_band_lu<R, true><<<nsys, kLuThreads, smem, st>>>(bd.Bd, bd.n, b, nb, K, z_dev, o, scratch);
    else
      k_band_lu<R, false><<<nsys, kLuThreads, smem, st>>>(bd.Bd, bd.n, b, nb, K, z_dev, o, scratch);
    FB_HIP(hipGetLastError());
  }
  size_t full = sizeof(cx<R>) * ((size_t)nb * nb + nb);
  bool ilds = full <= kLdsBudget;
  size_t ismem = ilds ? full : sizeof(cx<R>) * (size_t)nb;
  (void)hipFuncSetAttribute((const void*)k_block_invert<R, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  int nblk = nsys * K;
  ProfScope ps(FB_PROF_INVERT, st, 8.0 * 2.0 * nblk * (double)nb * nb * nb / 3.0);
  if (ilds)
    k_block_invert<R, true><<<2 * nblk, 256, ismem, st>>>(mats, nb, nblk);
  else
    k_block_invert<R, false><<<2 * nblk, 256, ismem, st>>>(mats, nb, nblk);
  FB_HIP(hipGetLastError());
  return 0;
}

template int launch_lu_impl<float>(const Band&, int, const c128*, c64*, int16_t*, int32_t*, c64*,
                                   c64*, hipStream_t);
template int launch_lu_impl<double>(const Band&, int, const c128*, c128*, int16_t*, int32_t*,
                                    c128*, c128*, hipStream_t);
template size_t lu_window_scratch<float>(int, int);
template size_t lu_window_scratch<double>(int, int);

}  // namespace fb
