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
};

template <typename R>
__device__ __forceinline__ cx<R> shifted_entry(const c128* __restrict__ Bd, int64_t n,
                                               int b, int64_t i, int64_t c, c128 z) {
  // A(i, c) of zI - B, padded with the identity beyond n
  if (i >= n || c >= n) return mk<R>(i == c ? (R)1 : (R)0, (R)0);
  int64_t d = i - c;
  c128 v;
  if (d >= 0) {
    if (d > b) return mk<R>(0, 0);
    c128 e = Bd[d * n + c];
    v = mk(-e.x, -e.y);
  } else {
    if (-d > b) return mk<R>(0, 0);
    c128 e = Bd[(-d) * n + i];
    v = mk(-e.x, e.y);  // -conj(B(c, i))
  }
  if (d == 0) {
    v.x += z.x;
    v.y = z.y;  // the diagonal of B is real
  }
  return mk<R>((R)v.x, (R)v.y);
}

template <typename R>
__global__ void __launch_bounds__(kLuThreads)
k_band_lu(const c128* __restrict__ Bd, int64_t n, int b, int nb, int K,
          const c128* __restrict__ zs, FactorOut<R> out, cx<R>* __restrict__ gwin,
          int use_lds) {
  extern __shared__ char lds_raw[];
  const int MR = b + 2, MC = 2 * b + 2;
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t npad = (int64_t)K * nb;
  const c128 z = zs[s];

  // LDS: phys[MR] int, idx[2][2nb] int, piv info, lvec[b+1] cx<R>, then window
  int* phys = reinterpret_cast<int*>(lds_raw);
  int* idx = phys + MR;                   // two perm buffers (block parity)
  int* pivp = idx + 4 * nb;               // [0] = pivot row of this step
  cx<R>* lvec = reinterpret_cast<cx<R>*>(lds_raw + ((sizeof(int) * (MR + 4 * nb + 4) + 15) & ~15));
  cx<R>* W = use_lds ? lvec + b + 1 : gwin + (size_t)s * MR * MC;

  cx<R>* mats = out.mats + (size_t)s * K * 5 * nb * nb;
  int16_t* permg = out.perm + (size_t)s * K * 2 * nb;
  const size_t bb = (size_t)nb * nb;

  // --- init: zero window, load rows 0..b, identity tables, zero block 0 Lh
  for (int e = t; e < MR * MC; e += blockDim.x) W[e] = mk<R>(0, 0);
  for (int e = t; e < MR; e += blockDim.x) phys[e] = e;
  for (int e = t; e < 2 * nb; e += blockDim.x) idx[e] = e;
  for (size_t e = t; e < 2 * bb; e += blockDim.x) mats[e] = mk<R>(0, 0);  // Lh11, Lh21 of block 0
  if (t == 0) out.info[s] = 0;
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

  int first_zero = 0;
  // running slots: row j sits in slot jr = j mod MR, column j in jcs = j mod MC;
  // an offset below MR (MC) needs at most one wrap
  int jr = 0, jcs = 0, k = 0, jj = 0;
  auto rslot = [&](int off) { int v = jr + off; return v >= MR ? v - MR : v; };
  auto cslot = [&](int off) { int v = jcs + off; return v >= MC ? v - MC : v; };
  for (int64_t j = 0; j < npad; ++j) {
    const int par = k & 1;
    int* idxk = idx + par * 2 * nb;
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
      // physical row of logical row j + r after the interchange
      cx<R> piv = W[(size_t)physp_old * MC + jc];
      cx<R> rp = cabs2(piv) > (R)0 ? cinv(piv) : mk<R>(0, 0);
      for (int r = t + 1; r <= nr; r += 64) {
        int pr = (r == bi) ? physj_old : phys[rslot(r)];
        cx<R> l = W[(size_t)pr * MC + jc] * rp;
        lvec[r - 1] = l;
        int wr = jj + r;  // window row of the block
        if (wr < nb)
          mats[((size_t)k * 5 + 0) * bb + (size_t)jj * nb + wr] = l;
        else
          mats[((size_t)k * 5 + 1) * bb + (size_t)jj * nb + (wr - nb)] = l;
      }
      if (t == 0) {
        phys[sj] = physp_old;
        phys[sp] = physj_old;
        int pw0 = jj + bi;
        int a = idxk[jj];
        idxk[jj] = idxk[pw0];
        idxk[pw0] = a;
        pivp[0] = pw0;
        if (!(cabs2(piv) > (R)0) && first_zero == 0) first_zero = (int)(j + 1);
      }
    }
    __syncthreads();

    // ---- phase B (all): U row, multiplier interchange, update, entering row
    const int pw = pivp[0];
    const int prj = phys[jr];
    {
      // U row j: columns k nb .. k nb+3nb-1 of blocks U(k,k), U(k,k+1), U(k,k+2)
      for (int e = t; e < 3 * nb; e += blockDim.x) {
        int co = e - jj;  // column offset from j
        cx<R> v = mk<R>(0, 0);
        if (co >= 0 && co <= nc) v = W[(size_t)prj * MC + cslot(co)];
        int which = 2 + e / nb;
        mats[((size_t)k * 5 + which) * bb + (size_t)(e % nb) * nb + jj] = v;
      }
      // keep Lh in the form P A = Lh U: earlier multipliers follow the rows
      if (pw != jj) {
        for (int c = t; c < jj; c += blockDim.x) {
          size_t a0 = (jj < nb) ? ((size_t)k * 5 + 0) * bb + (size_t)c * nb + jj
                                : ((size_t)k * 5 + 1) * bb + (size_t)c * nb + (jj - nb);
          size_t a1 = (pw < nb) ? ((size_t)k * 5 + 0) * bb + (size_t)c * nb + pw
                                : ((size_t)k * 5 + 1) * bb + (size_t)c * nb + (pw - nb);
          cx<R> va = mats[a0];
          mats[a0] = mats[a1];
          mats[a1] = va;
        }
      }
      // rank-one update of rows j+1..last, columns j+1..cend
      for (int e = t; e < nr * nc; e += blockDim.x) {
        int ro = e / nc, co = e - ro * nc;
        int cs = cslot(co + 1);
        size_t a = (size_t)phys[rslot(ro + 1)] * MC + cs;
        cx<R> u = W[(size_t)prj * MC + cs];
        cx<R> l = lvec[ro];
        cx<R> v = W[a];
        v.x -= l.x * u.x - l.y * u.y;
        v.y -= l.x * u.y + l.y * u.x;
        W[a] = v;
      }
      // column j+2b+1 enters: zero it in rows j+1..j+b (out of their band)
      {
        int cs = cslot(2 * b + 1);
        for (int r = t; r < b; r += blockDim.x) W[(size_t)phys[rslot(r + 1)] * MC + cs] = mk<R>(0, 0);
      }
      // row j+b+1 enters (columns j+1 .. j+2b+1)
      int64_t inew = j + b + 1;
      if (inew < npad) {
        int pr = phys[rslot(b + 1)];
        for (int e = t; e <= 2 * b; e += blockDim.x) {
          int64_t c = j + 1 + e;
          cx<R> v = mk<R>(0, 0);
          if (c < npad) v = shifted_entry<R>(Bd, n, b, inew, c, z);
          W[(size_t)pr * MC + cslot(1 + e)] = v;
        }
      }
      if (jj == nb - 1) {
        // block k complete: publish its permutation, prepare block k+1
        for (int e = t; e < 2 * nb; e += blockDim.x) {
          permg[(size_t)k * 2 * nb + e] = (int16_t)idxk[e];
          idx[(par ^ 1) * 2 * nb + e] = e;
        }
        if (k + 1 < K)
          for (size_t e = t; e < 2 * bb; e += blockDim.x)
            mats[((size_t)(k + 1) * 5) * bb + e] = mk<R>(0, 0);
      }
    }
    __syncthreads();
    jr = rslot(1);
    jcs = cslot(1);
    if (++jj == nb) {
      jj = 0;
      ++k;
    }
  }
  if (t == 0 && first_zero) out.info[s] = first_zero;
}

// In-place inverses of the unit lower Lh11 and the upper U(k,k) of every
// block: one workgroup per (system, block, which).  Column recurrences on the
// already inverted part (trailing part for L, leading part for U):
//   L = [1 0; l L22]:      L^{-1} column j below the diagonal = -L22^{-1} l
//   U = [U11 u; 0 ujj]:    U^{-1} column j above the diagonal = -U11^{-1} u / ujj
// The matrix is staged in LDS when it fits, else worked on in place in global
// memory; only the column being replaced is copied aside.
template <typename R>
__global__ void __launch_bounds__(256)
k_block_invert(cx<R>* __restrict__ mats, int b, int nblk, int use_lds) {
  extern __shared__ char lds_raw[];
  const int g = blockIdx.x;
  const int blk = g >> 1, which = g & 1;  // 0: Lh11 (slot 0), 1: U(k,k) (slot 2)
  if (blk >= nblk) return;
  cx<R>* M = mats + ((size_t)blk * 5 + (which ? 2 : 0)) * b * b;
  cx<R>* xv = reinterpret_cast<cx<R>*>(lds_raw);
  cx<R>* A = use_lds ? xv + b : M;
  const int t = threadIdx.x;
  const int bb = b * b;
  if (use_lds) {
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
  if (use_lds)
    for (int e = t; e < bb; e += blockDim.x) M[e] = A[e];
}

template <typename R>
static size_t lu_lds_head_bytes(int b) {
  const int nb = block_size(b);
  size_t head = (sizeof(int) * (size_t)((b + 2) + 4 * nb + 4) + 15) & ~(size_t)15;
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
                   int32_t* info, cx<R>* scratch, hipStream_t st) {
  const int b = bd.b;
  const int nb = block_size(b);
  const int K = (int)((bd.n + nb - 1) / nb);
  FactorOut<R> o{mats, perm, info};
  bool lds = lu_lds_bytes<R>(b) <= kLdsBudget;
  size_t smem = lds ? lu_lds_bytes<R>(b) : lu_lds_head_bytes<R>(b);
  (void)hipFuncSetAttribute((const void*)k_band_lu<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLdsBudget);
  (void)hipGetLastError();
  {
    ProfScope ps(FB_PROF_LU, st, 16.0 * (double)bd.n * b * b * nsys);
    k_band_lu<R><<<nsys, kLuThreads, smem, st>>>(bd.Bd, bd.n, b, nb, K, z_dev, o, scratch,
                                                  lds ? 1 : 0);
    FB_HIP(hipGetLastError());
  }
  size_t full = sizeof(cx<R>) * ((size_t)nb * nb + nb);
  bool ilds = full <= kLdsBudget;
  size_t ismem = ilds ? full : sizeof(cx<R>) * (size_t)nb;
  (void)hipFuncSetAttribute((const void*)k_block_invert<R>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  (void)hipGetLastError();
  int nblk = nsys * K;
  ProfScope ps(FB_PROF_INVERT, st, 8.0 * 2.0 * nblk * (double)nb * nb * nb / 3.0);
  k_block_invert<R><<<2 * nblk, 256, ismem, st>>>(mats, nb, nblk, ilds ? 1 : 0);
  FB_HIP(hipGetLastError());
  return 0;
}

template int launch_lu_impl<float>(const Band&, int, const c128*, c64*, int16_t*, int32_t*, c64*,
                                   hipStream_t);
template int launch_lu_impl<double>(const Band&, int, const c128*, c128*, int16_t*, int32_t*,
                                    c128*, hipStream_t);
template size_t lu_window_scratch<float>(int, int);
template size_t lu_window_scratch<double>(int, int);

}  // namespace fb
