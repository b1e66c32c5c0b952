// Batched complex FP64 GEMMs on FP64 MFMA: the Gram, projection and basis
// products of the orthonormalisation and Rayleigh-Ritz step (Algorithm
// alg:FEAST: Q^H Q, Q^H (B Q), Q W), and the block updates of the blocked
// Cholesky factorisation and triangular inverse of the reduced matrices.
//
// One workgroup of 4 waves computes one 64 x 64 tile of C over one
// contraction range.  The contraction advances in chunks of 16: each chunk
// of op(A) (64 x 16) and B (16 x 64) is loaded from HBM into registers one
// chunk ahead, stored to one of two LDS stages and consumed from LDS by the
// waves, each owning a 32 x 32 quarter of the tile as 2 x 2 MFMA tiles of
// 16 x 16.  Complex products take three real 16x16x4 FP64 MFMAs in Gauss
// form (p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi); real p1 - p2,
// imaginary p3 - p1 - p2).
#include <algorithm>

#include "gemm64.h"
#include "prof.h"

namespace fb {

typedef double gd4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int TT = kGemmTile;  // output tile
constexpr int KC = 16;         // contraction chunk per LDS stage
constexpr int PK = KC + 1;     // padded row length of the [row][k] layouts
constexpr int NTH = 256;       // threads per workgroup
constexpr int STAGE = TT * PK; // complex elements per operand per stage

__device__ __forceinline__ gd4 mfma64(double a, double b, gd4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// workgroup -> (product, tile row, tile column, split); jobs of one product
// are numbered split-major, then tile row, then tile column, and dealt so
// that each XCD runs a contiguous range (neighbouring tiles share operand
// strips in that XCD's L2).  The grid is a multiple of 8 (8 per workgroups),
// which makes the map a bijection onto 0 .. 8 per - 1.
__device__ __forceinline__ int gemm_remap(int bid, int nwg) {
  const int per = (nwg + 7) / 8;
  return (bid % 8) * per + bid / 8;
}
}  // namespace

template <bool TA>
__global__ void __launch_bounds__(NTH)
k_zgemm64(const GemmProb* __restrict__ probs, int nprob, int nwg) {
  extern __shared__ __align__(16) char lds_raw[];
  c128* lds = reinterpret_cast<c128*>(lds_raw);  // 2 stages x (op(A), B)
  const int job = gemm_remap(blockIdx.x, nwg);
  if (job >= nwg) return;
  // product of this job: the last descriptor with tile0 <= job
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile0 <= job) lo = mid;
    else hi = mid - 1;
  }
  const GemmProb& P = probs[lo];
  const int loc = job - P.tile0;
  const int per_split = P.tm * P.tn;
  const int s = loc / per_split;
  const int ti = (loc % per_split) / P.tn, tj = loc % P.tn;
  if (s >= P.ksplit) return;
  if (P.herm && ti > tj) return;
  const int M = P.M, N = P.N, K = P.K;
  const int i0 = ti * TT, j0 = tj * TT;
  // contraction range of this tile and split
  int kb = P.a_upper ? i0 : 0;
  int ke = P.b_upper ? min(K, j0 + TT) : K;
  if (P.ksplit > 1) {
    const int len = ke - kb;
    const int chunk = ((len + P.ksplit - 1) / P.ksplit + KC - 1) / KC * KC;
    const int b2 = kb + s * chunk;
    ke = min(ke, b2 + chunk);
    kb = b2;
  }
  const c128* A = P.A;  // B may alias C (in-place panel updates): no restrict
  const c128* B = P.B;
  const int64_t lda = P.lda, ldb = P.ldb;

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w & 1, wc = w >> 1;
  const int li = lane & 15, lk = lane >> 4;

  // global -> register loads of one chunk (branch-free: an out-of-range
  // element reads the operand's first element and is zeroed when stored),
  // issued one chunk ahead of the products.  The chunk's k-steps are not
  // unrolled and the stores select values, which keeps every operand in
  // registers (112 VGPRs, two waves per SIMD, no scratch)
  struct Regs {
    c128 a[4], b[4];
  };
  // element coordinates of this thread's loads (validity recomputed at the store)
  auto a_ok = [&](int kc, int q) {
    if (TA) return (i0 + (t >> 2)) < M && kc + (t & 3) * 4 + q < ke;
    return (i0 + (t & 15) * 4 + q) < M && kc + (t >> 4) < ke;
  };
  auto b_ok = [&](int kc, int q) { return (j0 + (t >> 2)) < N && kc + (t & 3) * 4 + q < ke; };
  auto issue = [&](Regs& R, int kc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t off;
      if (TA) off = (int64_t)(i0 + (t >> 2)) * lda + kc + (t & 3) * 4 + q;
      else off = (int64_t)(kc + (t >> 4)) * lda + i0 + (t & 15) * 4 + q;
      R.a[q] = gld(A + (a_ok(kc, q) ? off : 0));
      const int64_t offb = (int64_t)(j0 + (t >> 2)) * ldb + kc + (t & 3) * 4 + q;
      R.b[q] = gld(B + (b_ok(kc, q) ? offb : 0));
    }
  };
  auto store = [&](const Regs& R, int stg, int kc) {
    c128* As = lds + stg * 2 * STAGE;
    c128* Bs = As + STAGE;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // selects on values (a select of lvalues would put R in memory)
      const bool oa = a_ok(kc, q), ob = b_ok(kc, q);
      const c128 va = mk(oa ? R.a[q].x : 0.0, oa ? R.a[q].y : 0.0);
      const c128 vb = mk(ob ? R.b[q].x : 0.0, ob ? R.b[q].y : 0.0);
      if (TA) As[(t >> 2) * PK + (t & 3) * 4 + q] = va;
      else As[(t >> 4) * TT + (t & 15) * 4 + q] = va;
      Bs[(t >> 2) * PK + (t & 3) * 4 + q] = vb;
    }
  };

  gd4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) p1[a][b][r] = p2[a][b][r] = p3[a][b][r] = 0.0;
  auto compute = [&](int stg) {
    const c128* As = lds + stg * 2 * STAGE;
    const c128* Bs = As + STAGE;
#pragma unroll 1
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = 4 * kk + lk;
      double ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int i = 32 * wr + 16 * rt + li;
        const c128 a = TA ? As[i * PK + k] : As[k * TT + i];
        ar[rt] = a.x;
        ai[rt] = TA ? -a.y : a.y;
        as[rt] = ar[rt] + ai[rt];
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const int j = 32 * wc + 16 * ct + li;
        const c128 b = Bs[j * PK + k];
        br[ct] = b.x;
        bi[ct] = b.y;
        bs[ct] = b.x + b.y;
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          p1[rt][ct] = mfma64(ar[rt], br[ct], p1[rt][ct]);
          p2[rt][ct] = mfma64(ai[rt], bi[ct], p2[rt][ct]);
          p3[rt][ct] = mfma64(as[rt], bs[ct], p3[rt][ct]);
        }
    }
  };

  const int nch = ke > kb ? (ke - kb + KC - 1) / KC : 0;
  Regs R0;
  if (nch > 0) {
    issue(R0, kb);
    store(R0, 0, kb);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int stg = c & 1;
    if (c + 1 < nch) issue(R0, kb + (c + 1) * KC);
    compute(stg);
    if (c + 1 < nch) store(R0, stg ^ 1, kb + (c + 1) * KC);
    __syncthreads();
  }

  // epilogue: register r of lane l holds row (l / 16) + 4 r, column l % 16
  const c128 al = P.alpha;
  const bool split = P.ksplit > 1;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 32 * wr + 16 * rt + lk + 4 * r;
        const int j = j0 + 32 * wc + 16 * ct + li;
        if (i >= M || j >= N) continue;
        const double x1 = p1[rt][ct][r], x2 = p2[rt][ct][r], x3 = p3[rt][ct][r];
        const c128 v = mk(x1 - x2, x3 - x1 - x2);
        if (split) {
          gst(P.part + ((int64_t)s * N + j) * M + i, v);
        } else {
          c128* cp = P.C + (int64_t)j * P.ldc + i;
          c128 o = al * v;
          if (P.beta) o = o + gld(cp);
          gst(cp, o);
        }
      }
}

// Split sums (in split order) with alpha and beta, and the Hermitian mirror
// (herm == 2): C(j, i) = conj(C(i, j)) for i < j, real diagonal.
__global__ void __launch_bounds__(256)
k_zgemm64_finish(const GemmProb* __restrict__ probs) {
  const GemmProb& P = probs[blockIdx.y];
  if (P.ksplit <= 1 && P.herm != 2) return;
  const int M = P.M, N = P.N;
  const int64_t tot = (int64_t)M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / M), i = (int)(e - (int64_t)j * M);
    if (P.herm && i > j) continue;
    c128* cp = P.C + (int64_t)j * P.ldc + i;
    c128 v;
    if (P.ksplit > 1) {
      v = mk(0.0, 0.0);
      for (int s = 0; s < P.ksplit; ++s) v = v + gld(P.part + ((int64_t)s * N + j) * M + i);
      v = P.alpha * v;
      if (P.beta) v = v + gld(cp);
    } else {
      v = gld(cp);
    }
    if (P.herm == 2 && i == j) v.y = 0.0;
    gst(cp, v);
    if (P.herm == 2 && i < j) gst(P.C + (int64_t)i * P.ldc + j, cconj(v));
  }
}

static const size_t kGemmLds = 2 * 2 * STAGE * sizeof(c128);

static double gemm_work(const GemmProb& p) {
  const double M = p.M, N = p.N, K = p.K;
  if (p.herm) return 8.0 * K * M * (M + 1) / 2;
  if (p.a_upper) return 8.0 * N * M * (M + 1) / 2;
  if (p.b_upper) return 8.0 * M * N * (N + 1) / 2;
  return 8.0 * M * N * K;
}

size_t gemm_part_bytes(const GemmProb& p) {
  return p.ksplit > 1 ? (size_t)p.ksplit * p.M * p.N * sizeof(c128) : 0;
}

int gemm_choose_split(const std::vector<GemmProb>& probs, int target_wgs) {
  long tiles = 0;
  for (const GemmProb& p : probs) {
    const long tm = (p.M + TT - 1) / TT, tn = (p.N + TT - 1) / TT;
    tiles += p.herm ? tm * (tm + 1) / 2 : tm * tn;
  }
  if (tiles <= 0) return 1;
  int s = (int)((target_wgs + tiles - 1) / tiles);
  return std::max(1, std::min(s, 16));
}

static void gemm_set_attr() {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_zgemm64<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
    (void)hipFuncSetAttribute((const void*)k_zgemm64<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
    (void)hipGetLastError();
    attr = true;
  }
}

int gemm_prepare(GemmProb* v, int nprob, GemmBatch& b) {
  if (nprob > kGemmMaxProbs) return FB_ERR_INTERNAL;
  b = GemmBatch{};
  b.nprob = nprob;
  b.transa = -1;
  for (int q = 0; q < nprob; ++q) {
    GemmProb& p = v[q];
    if (p.ksplit < 1) p.ksplit = 1;
    if (p.M < 0 || p.N < 0 || p.K < 0) return FB_ERR_INTERNAL;
    if (p.ksplit > 1 && (p.a_upper || p.b_upper || !p.part)) return FB_ERR_INTERNAL;
    if (p.herm && p.M != p.N) return FB_ERR_INTERNAL;
    if (p.M > 0 && p.N > 0) {  // one form per batch (empty products take no part)
      if (b.transa < 0) b.transa = p.transa;
      if (p.transa != b.transa) return FB_ERR_INTERNAL;
    }
    p.tm = (p.M + TT - 1) / TT;
    p.tn = (p.N + TT - 1) / TT;
    p.tile0 = b.nwg;
    b.nwg += p.tm * p.tn * p.ksplit;
    b.work += gemm_work(p);
    b.finish = b.finish || p.ksplit > 1 || p.herm == 2;
  }
  if (b.transa < 0) b.transa = 0;
  return 0;
}

int gemm_launch(const GemmProb* probs_dev, const GemmBatch& b, hipStream_t st) {
  if (b.nwg <= 0) return 0;
  gemm_set_attr();
  {
    ProfScope ps(FB_PROF_GEMM, st, b.work);
    // a multiple of 8 workgroups, so that the XCD remapping is a bijection
    if (b.transa)
      k_zgemm64<true><<<8 * ((b.nwg + 7) / 8), NTH, kGemmLds, st>>>(probs_dev, b.nprob, b.nwg);
    else
      k_zgemm64<false><<<8 * ((b.nwg + 7) / 8), NTH, kGemmLds, st>>>(probs_dev, b.nprob, b.nwg);
    FB_HIP(hipGetLastError());
  }
  if (b.finish) {
    k_zgemm64_finish<<<dim3(512, (unsigned)b.nprob), 256, 0, st>>>(probs_dev);
    FB_HIP(hipGetLastError());
  }
  return 0;
}

int gemm_batched(std::vector<GemmProb> probs, GemmProb* probs_dev, hipStream_t st) {
  std::vector<GemmProb> live;
  for (GemmProb& p : probs)
    if (p.M > 0 && p.N > 0) live.push_back(p);
  for (size_t c0 = 0; c0 < live.size(); c0 += kGemmMaxProbs) {
    const int nc = (int)std::min(live.size() - c0, (size_t)kGemmMaxProbs);
    GemmBatch b;
    FB_TRY(gemm_prepare(live.data() + c0, nc, b));
    FB_HIP(hipMemcpyAsync(probs_dev, live.data() + c0, sizeof(GemmProb) * nc,
                          hipMemcpyHostToDevice, st));
    FB_TRY(gemm_launch(probs_dev, b, st));
    if (c0 + nc < live.size()) FB_HIP(hipStreamSynchronize(st));  // descriptors reused
  }
  return 0;
}

}  // namespace fb
