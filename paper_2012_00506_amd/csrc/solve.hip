// Multi-right-hand-side solves with the block form of the band LU factors.
// Every sweep step is one set of independent products of blocks formed once
// per factorisation (M = Lh21 Lh11^{-1}, Q = U(k,k)^{-1} Lh11^{-1},
// G1 = U(k,k)^{-1} U(k,k+1), G2 = U(k,k)^{-1} U(k,k+2)), so that a step
// waits for the previous one only once.
//
// N: x = A^{-1} y.  Forward, block k on the window rows kb .. kb+2b-1:
//      z = P y_win; v_k = Q z_top; carry = z_bot - M z_top
//    (v_k = U(k,k)^{-1} Lh11^{-1} z_top).
//    Backward: x_k = v_k - G1 x_{k+1} - G2 x_{k+2}
//    (= U(k,k)^{-1} (Lh11^{-1} z_top - U(k,k+1) x_{k+1} - U(k,k+2) x_{k+2})).
// H: x = A^{-H} y.  Forward with U^H, in u_k = U(k,k)^H w_k:
//      u_k = y_k - G1(k-1)^H u_{k-1} - G2(k-2)^H u_{k-2}
//    (w_k = U(k,k)^{-H} (y_k - U(k-1,k)^H w_{k-1} - U(k-2,k)^H w_{k-2})).
//    Backward, k descending on the window [u_k ; carry]:
//      top = Q^H u_k - M^H carry; x_win = P^T [top ; carry]
//    (top = Lh11^{-H} w_k - M^H carry; rows kb+b .. kb+2b-1 of x_win are
//    final, rows kb .. kb+b-1 carry on).
// One workgroup per job (system, direction, tile of T columns); the tile's
// window and carries live in LDS.  Inputs and outputs are complex128; the
// arithmetic is in R (float: complex64 path, double: complex128 path).
#include "solve_kernel.h"
#include "tune.h"

namespace fb {
// the kernels live in solve_f32.hip / solve_f64.hip
extern template int launch_variant<float>(int, const c64*, const c64*, const int16_t*, int64_t,
                                          int, int, const SolveJob*, hipStream_t, const int32_t*);
extern template int launch_variant<double>(int, const c128*, const c128*, const int16_t*, int64_t,
                                           int, int, const SolveJob*, hipStream_t, const int32_t*);
}  // namespace fb

namespace fb {

// ---------------------------------------------------------------- dispatch
template <typename R>
int solve_tile(int b) {
  return variant_tile(tuned_variant(sizeof(R), block_size(b)));
}

template <typename R>
int launch_solve_jobs(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n,
                      int b, int njobs, const SolveJob* jobs_dev, double work, hipStream_t st,
                      const int32_t* gate) {
  if (njobs <= 0) return 0;
  if (sizeof(R) == 4 && matsT == nullptr) return FB_ERR_INTERNAL;
  ProfScope ps(FB_PROF_SOLVE, st, work);
  const int nb = block_size(b);
  return launch_variant<R>(tuned_variant(sizeof(R), nb), mats, matsT, perm, n, nb, njobs,
                           jobs_dev, st, gate);
}

template int launch_solve_jobs<float>(const c64*, const c64*, const int16_t*, int64_t, int, int,
                                      const SolveJob*, double, hipStream_t, const int32_t*);
template int launch_solve_jobs<double>(const c128*, const c128*, const int16_t*, int64_t, int,
                                       int, const SolveJob*, double, hipStream_t, const int32_t*);
template int solve_tile<float>(int);
template int solve_tile<double>(int);

// ---------------------------------------------------------------- residual
// r = y - (zz x - B x) in FP64 for the columns of a job (zz = z for A x = y,
// conj(z) for A^H x = y), with B in block-tridiagonal form:
// (B x)_k = B(k,k-1) x_{k-1} + B(k,k) x_k + B(k,k+1) x_{k+1}, each an NB x NB
// by NB x T product on f64 MFMA (three real products per complex one), one
// wave per 16 x 16 output tile.  x blocks roll through three LDS slots and a
// fourth holds y_k, then r_k; tiles enter and leave global memory with thread
// e on row e % NB, column e / NB, so that a wave moves whole column runs.
//
// A wave's share of the three products is a fixed list of 2 NB/16 + 1
// chunks of 16 B columns (the triangles of B(k,k-1) and B(k,k+1) outside
// the band are skipped).  Its B fragments are loaded chunk by chunk RD chunks
// ahead of the MFMAs that use them, across block rows and barriers, so that
// no product waits for its first fragment.  The blocks B(0,-1) and
// B(K-1,K) are zero, as are the x slots beyond the ends, so every block row
// runs the same list.  Per (job, column): sum |r|^2 and sum |y|^2.
template <int NB, int T>
__global__ void __launch_bounds__(NB * 4 * (T / 16))
k_shift_residual(const c128* __restrict__ Bblk, int64_t n, int K, const ResJob* __restrict__ jobs,
                 int njobs, double* __restrict__ part, const int32_t* __restrict__ gate) {
  constexpr int LDT = T + 1;    // LDS row of a slot
  constexpr int SL = NB * LDT;  // one slot
  constexpr int NTH = NB * 4 * (T / 16);
  constexpr int RX = NB * T / NTH;  // tile elements per thread
  constexpr int NRW = NB / 16;
  constexpr int L = 2 * NRW + 1;    // chunks per block row and wave
  // chunks of fragments in flight: two where the registers hold them
  // without spilling (checked per block size), else one
  constexpr int RD = (NB <= 32 || NB == 64) ? 2 : 1;
  extern __shared__ __align__(16) char lds_raw[];
  c128* X = reinterpret_cast<c128*>(lds_raw);  // 3 slots of x blocks
  c128* Yr = X + 3 * SL;                       // y_k, overwritten by r_k
  const int job = remap_job(blockIdx.x, njobs);
  if (job >= njobs) return;
  const ResJob jb = jobs[job];
  if (gate && !gate[jb.grp]) return;  // the group has finished refining
  const c128* jx = jb.x;
  const c128* jy = jb.y;
  c128* jr = jb.r;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int w = __builtin_amdgcn_readfirstlane(wv % NRW);
  const int cb0 = __builtin_amdgcn_readfirstlane(16 * (wv / NRW));
  const int c0 = jb.col0;
  const int nc = jb.ncol;
  const size_t bb = (size_t)NB * NB;
  const c128 zz = jb.dir ? mk(jb.z.x, -jb.z.y) : jb.z;
  const int kq = lane >> 4;
  const int col = cb0 + (lane & 15);
  // chunk i of the list: product p (0: B(k,k-1), 1: B(k,k), 2: B(k,k+1))
  // over B columns 16 ch .. 16 ch + 15
  const int n0 = NRW - w;  // chunks of product 0
  auto chunk_p = [&](int i) { return i < n0 ? 0 : (i < n0 + NRW ? 1 : 2); };
  auto chunk_c = [&](int i) { return i < n0 ? w + i : (i < n0 + NRW ? i - n0 : i - n0 - NRW); };
  // fragment q of a chunk: B[16 w + lane % 16][16 ch + 4 q + lane / 16]
  struct Ch {
    c128 a[4];
  };
  const c128* Brow = Bblk + (size_t)(kq * NB + 16 * w + (lane & 15));
  auto cload = [&](Ch& f, int k, int i) {
    const c128* A = Brow + ((size_t)k * 3 + chunk_p(i)) * bb + (size_t)(16 * chunk_c(i)) * NB;
#pragma unroll
    for (int q = 0; q < 4; ++q) f.a[q] = gld(A + (size_t)(4 * q) * NB);
  };
  // tile element q of this thread: row e % NB, column e / NB (one column
  // per wave and q)
  auto erow = [&](int q) { return (t + q * NTH) % NB; };
  auto ecol = [&](int q) { return (t + q * NTH) / NB; };
  auto ok = [&](int k, int q) {
    const int64_t i = (int64_t)k * NB + erow(q);
    return k < K && i < n && ecol(q) < nc;
  };
  // branch-free loads (clamped address, zeroed when stored), issued one
  // block row ahead so that their latency overlaps the products
  auto tissue = [&](c128* v, const c128* base, int64_t ld, int k) {
#pragma unroll
    for (int q = 0; q < RX; ++q)
      v[q] = gld(base + (ok(k, q) ? (int64_t)(c0 + ecol(q)) * ld + (int64_t)k * NB + erow(q) : 0));
  };
  auto tstore = [&](const c128* v, c128* dst, int k) {
#pragma unroll
    for (int q = 0; q < RX; ++q) dst[erow(q) * LDT + ecol(q)] = ok(k, q) ? v[q] : mk(0.0, 0.0);
  };
  for (int e = t; e < SL; e += NTH) X[2 * SL + e] = mk(0.0, 0.0);  // x_{-1}
  c128 xr[RX], yv[RX];
  double rr[RX], yy[RX];
#pragma unroll
  for (int q = 0; q < RX; ++q) rr[q] = yy[q] = 0.0;
  Ch carry[RD];
#pragma unroll
  for (int i = 0; i < RD; ++i) cload(carry[i], 0, i);
  tissue(xr, jx, jb.ldx, 0);
  tstore(xr, X, 0);
  tissue(xr, jx, jb.ldx, 1);
  tissue(yv, jy, jb.ldy, 0);
  for (int k = 0; k < K; ++k) {
    tstore(xr, X + ((k + 1) % 3) * SL, k + 1);
    tstore(yv, Yr, k);
#pragma unroll
    for (int q = 0; q < RX; ++q)
      if (ok(k, q)) yy[q] += cabs2(yv[q]);
    __syncthreads();
    if (k + 2 <= K) tissue(xr, jx, jb.ldx, k + 2);
    if (k + 1 < K) tissue(yv, jy, jb.ldy, k + 1);
    const c128* Xk = X + (k % 3) * SL;
    const c128* Sp[3] = {X + ((k + 2) % 3) * SL, Xk, X + ((k + 1) % 3) * SL};
    const bool more = k + 1 < K;
    // (B x)_k over the chunk list, then r = y - zz x + B x
    Acc<double, 1> acc;
    acc.zero();
    Ch buf[L + RD];
#pragma unroll
    for (int i = 0; i < RD; ++i) buf[i] = carry[i];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      if (i + RD < L)
        cload(buf[i + RD], k, i + RD);
      else if (more)
        cload(buf[i + RD], k + 1, i + RD - L);
      const int p = chunk_p(i), ch = chunk_c(i);
      const c128* bp = (p == 0 ? Sp[0] : (p == 1 ? Sp[1] : Sp[2])) + (16 * ch + kq) * LDT + col;
      c128 bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = bp[4 * q * LDT];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double ar = buf[i].a[q].x, ai = buf[i].a[q].y;
        acc.p1[0] = MF<double>::mma(ar, bv[q].x, acc.p1[0]);
        acc.p2[0] = MF<double>::mma(ai, bv[q].y, acc.p2[0]);
        acc.p3[0] = MF<double>::mma(ar + ai, bv[q].x + bv[q].y, acc.p3[0]);
      }
    }
#pragma unroll
    for (int i = 0; i < RD; ++i) carry[i] = buf[L + i];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + MF<double>::row(lane, r);
      c128* p = Yr + row * LDT + col;
      *p = *p - zz * Xk[row * LDT + col] + acc.get(0, r);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RX; ++q) {
      if (!ok(k, q)) continue;
      const c128 v = Yr[erow(q) * LDT + ecol(q)];
      gst(jr + (int64_t)(c0 + ecol(q)) * jb.ldr + (int64_t)k * NB + erow(q), v);
      rr[q] += cabs2(v);
    }
  }
  // column sums in a fixed order: per-element partial sums through LDS (the
  // x slots are free), then one thread per column adds its NB rows
  __syncthreads();
  double* red = reinterpret_cast<double*>(X);  // 2 x T columns x NB rows
#pragma unroll
  for (int q = 0; q < RX; ++q) {
    const int e = t + q * NTH;
    red[e] = rr[q];
    red[NB * T + e] = yy[q];
  }
  __syncthreads();
  if (t < T) {
    double sr = 0.0, sy = 0.0;
    for (int i = 0; i < NB; ++i) {
      sr += red[t * NB + i];
      sy += red[NB * T + t * NB + i];
    }
    part[((size_t)job * 32 + t) * 2] = sr;
    part[((size_t)job * 32 + t) * 2 + 1] = sy;
  }
}

// per group: ratio = max over its columns of sqrt(sum|r|^2 / sum|y|^2)
// (columns with y = 0 count as converged when r = 0), and the decision of
// the next refinement pass (RefineCtl)
__global__ void k_refine_decide(const double* __restrict__ part, int njobs,
                                const ResJob* __restrict__ jobs, RefineCtl ctl) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const int g = jobs[j].grp;
  if (ctl.gate && !ctl.gate[g]) return;
  double mx = 0.0;
  for (int c = 0; c < jobs[j].ncol; ++c) {
    double rr = part[((size_t)j * 32 + c) * 2], yy = part[((size_t)j * 32 + c) * 2 + 1];
    double q = yy > 0.0 ? sqrt(rr / yy) : (rr > 0.0 ? 1e300 : 0.0);
    if (!(q <= mx)) mx = q;  // NaN propagates
  }
  const double prev = ctl.ratio[g];
  ctl.ratio[g] = mx;
  if (ctl.pass == 0) ctl.npass[g] = 0;
  const bool more = ctl.ir && !(mx <= ctl.ir_tol) && ctl.pass < ctl.max_pass &&
                    (ctl.pass == 0 || mx < 0.5 * prev);
  ctl.flag[g] = more ? 1 : 0;
  if (more) ctl.npass[g] = ctl.pass + 1;
}

size_t residual_part_doubles(int64_t n, int njobs) {
  (void)n;
  return (size_t)njobs * 32 * 2;
}

// residual jobs carry up to 32 columns; blocks of 128 rows use 16-column
// tiles (LDS), the others 32
template <int NB>
static int launch_res_nb(const Band& bd, int njobs, const ResJob* jobs_dev, double* part,
                         const int32_t* gate, hipStream_t st) {
  constexpr int T = NB <= 64 ? 32 : 16;
  size_t smem = (size_t)4 * NB * (T + 1) * sizeof(c128);
  (void)hipFuncSetAttribute((const void*)k_shift_residual<NB, T>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
  for (int j0 = 0; j0 < njobs; j0 += 1 << 20) {
    int nj = njobs - j0 < (1 << 20) ? njobs - j0 : (1 << 20);
    int grid = 8 * ((nj + 7) / 8);
    k_shift_residual<NB, T><<<grid, NB * 4 * (T / 16), smem, st>>>(
        bd.Bblk, bd.n, bd.K, jobs_dev + j0, nj, part + (size_t)j0 * 64, gate);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

int residual_cols(int nb) { return nb <= 64 ? 32 : 16; }

int launch_residual_jobs(const Band& bd, int njobs, const ResJob* jobs_dev, double* part,
                         const RefineCtl& ctl, double work, hipStream_t st) {
  if (njobs <= 0) return 0;
  ProfScope ps(FB_PROF_RESID, st, work);
  int rc;
  const int32_t* gate = ctl.gate;
  switch (bd.nb) {
    case 16: rc = launch_res_nb<16>(bd, njobs, jobs_dev, part, gate, st); break;
    case 32: rc = launch_res_nb<32>(bd, njobs, jobs_dev, part, gate, st); break;
    case 48: rc = launch_res_nb<48>(bd, njobs, jobs_dev, part, gate, st); break;
    case 64: rc = launch_res_nb<64>(bd, njobs, jobs_dev, part, gate, st); break;
    case 80: rc = launch_res_nb<80>(bd, njobs, jobs_dev, part, gate, st); break;
    case 96: rc = launch_res_nb<96>(bd, njobs, jobs_dev, part, gate, st); break;
    case 112: rc = launch_res_nb<112>(bd, njobs, jobs_dev, part, gate, st); break;
    case 128: rc = launch_res_nb<128>(bd, njobs, jobs_dev, part, gate, st); break;
    default: return FB_ERR_INTERNAL;
  }
  if (rc) return rc;
  k_refine_decide<<<(njobs + 255) / 256, 256, 0, st>>>(part, njobs, jobs_dev, ctl);
  FB_HIP(hipGetLastError());
  return 0;
}

}  // namespace fb
