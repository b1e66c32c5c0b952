// Blocked Cholesky and triangular inverse of batched Hermitian matrices.
#pragma once
#include <vector>

#include "gemm64.h"

namespace fb {

// One matrix of the batch.
struct CholProb {
  c128* G;           // m x m, leading dimension ld: in, the upper triangle of
                     // G; out, R (G = R^H R) in the upper triangle (the strict
                     // lower triangle is left as it was)
  int64_t ld;
  c128* T;           // out: D R^{-1} (upper, zero below), leading dimension ldt
  int64_t ldt;
  c128* Dinv;        // scratch: ceil(m/64) blocks of 64 x 64
  c128* P;           // scratch: m x 64 (leading dimension m)
  const double* rowscale;  // D = diag(rowscale), or null for D = I
  int32_t* info;     // out: 0, or the first column (1-based) whose pivot
                     // r_jj^2 was not above piv_min
  int32_t m;
  int32_t pad_;
};

// GEMM descriptors chol_inverse needs (device area gdev, gcap entries).
size_t chol_gemm_descs(int nprob, int m_max);
int chol_inverse(const std::vector<CholProb>& probs, CholProb* probs_dev, GemmProb* gdev,
                 size_t gcap, double piv_min, hipStream_t st);

}  // namespace fb
