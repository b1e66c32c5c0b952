// Batched complex FP64 GEMMs on FP64 MFMA (Rayleigh-Ritz, orthonormalisation
// and the blocked Cholesky / triangular inverse that serve them).
#pragma once
#include <vector>

#include "fb_internal.h"

namespace fb {

// One product C = beta C + alpha op(A) B of a batch.  op(A) is A (M x K,
// leading dimension lda) or A^H (A is K x M); B is K x N; C is M x N; all
// column-major complex128.  beta is 0 (C not read) or 1.
//  herm    op(A) B is Hermitian (A^H A-like products): only the 64 x 64
//          tiles on or above the diagonal are computed; herm_finish mirrors
//  a_upper op(A) is upper triangular (entries below the diagonal are never
//          read): the contraction of row tile i starts at 64 i
//  b_upper B is upper triangular: column tile j stops at 64 (j + 1)
// Long contractions (op(A) = A^H with K far above M, N) are split into
// ksplit ranges whose partial tiles go to part (ksplit x M x N per product,
// summed in range order by herm_finish / split_finish, so the result does not
// depend on the launch).
struct GemmProb {
  const c128* A;
  const c128* B;
  c128* C;
  c128* part;
  int64_t lda, ldb, ldc;
  c128 alpha;
  int32_t M, N, K;
  int32_t transa;   // 1: op(A) = A^H
  int32_t beta;     // 0 or 1
  int32_t herm, a_upper, b_upper;
  int32_t ksplit;   // >= 1
  int32_t tm, tn;   // tiles (filled by the launcher)
  int32_t tile0;    // first workgroup of this product (filled by the launcher)
  int32_t pad_;
};

constexpr int kGemmTile = 64;
constexpr int kGemmMaxProbs = 256;

// Workspace of the split-K partial tiles of a batch (bytes), for the split
// the launcher will choose.
size_t gemm_part_bytes(const GemmProb& p);
// Choose ksplit for a long A^H B contraction so that the batch has enough
// workgroups; part must then hold gemm_part_bytes(p) bytes.
int gemm_choose_split(const std::vector<GemmProb>& probs, int target_wgs);

// probs_dev: device copy area for up to kGemmMaxProbs descriptors.
int gemm_batched(std::vector<GemmProb> probs, GemmProb* probs_dev, hipStream_t st);

// Two-phase form for sequences of small batches (blocked factorisations):
// gemm_prepare fills the launch fields of one batch (products with an empty
// C are given no workgroups) and returns what gemm_launch needs; the
// descriptors of many batches can then be copied to the device at once.
struct GemmBatch {
  int nprob = 0;
  int transa = 0;  // every product of a batch has the same form
  int nwg = 0;
  double work = 0.0;
  bool finish = false;
};
int gemm_prepare(GemmProb* probs, int nprob, GemmBatch& b);
int gemm_launch(const GemmProb* probs_dev, const GemmBatch& b, hipStream_t st);

}  // namespace fb
