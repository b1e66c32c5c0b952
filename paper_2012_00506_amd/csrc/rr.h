// Rayleigh-Ritz support kernels (host launch wrappers).
#pragma once
#include <algorithm>

#include <vector>

#include "fb_internal.h"

namespace fb {

struct JacobiJob {
  int32_t m;
  int32_t pad_;
  c128* A;        // in: Hermitian matrix (destroyed)
  int64_t lda;
  c128* V;        // scratch m x m (rotations accumulate here)
  int64_t ldv;
  c128* W;        // out: eigenvectors, columns in ascending eigenvalue order
  int64_t ldw;
  double* w;      // out: eigenvalues ascending
  int32_t* order; // scratch m
  int32_t* sweeps;// out (may be null)
};

int fill_zero(c128* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t st);

// Q += sum_p w_p X_p over the (node, direction) solutions of one slice, in
// the order p = 0, 1, ... (real B: Q += 2 Re(w_p X_p)).
constexpr int kMaxPairs = 128;
struct AccJob {
  c128* Q;
  int64_t ldq;
  const c128* X[kMaxPairs];
  int64_t ldx;
  c128 w[kMaxPairs];
  int32_t np;
  int32_t m;
  int32_t acc_real;
  int32_t init;  // 1: Q starts from zero (the first pairs of a sum), not read
};
int accumulate_pairs(const AccJob* jobs_dev, int njobs, int64_t n, int max_m, hipStream_t st);
int gather_cols(const void* src, int64_t lds, bool real_src, c128* dst, int64_t ldd,
                int64_t rows, int cols, const int32_t* idx_dev, const double* scale_dev,
                hipStream_t st);
int store_cols(const c128* src, int64_t lds, void* dst, int64_t ldd, bool real_dst, int64_t rows,
               int cols, const int32_t* idx_dev, hipStream_t st);
int hermitize(c128* A, int m, int64_t lda, hipStream_t st);
int band_matmul(const Band& bd, const c128* X, int64_t ldx, c128* Y, int64_t ldy, int m,
                hipStream_t st);
size_t eig_resid_part_doubles(int64_t n, int m);
int eig_residuals(const Band& bd, const c128* X, int64_t ldx, const double* lam, int m,
                  double* part, double* res, hipStream_t st);
int launch_jacobi(int njobs, JacobiJob* jobs_dev, int max_sweeps, double tol, hipStream_t st);

// Parallel block Jacobi (many workgroups per matrix) for larger matrices:
// work holds block_jacobi_bytes(m) per job, dv_dev one device descriptor
// per job (kBjDescBytes), norms_dev 2 doubles per job.  Synchronises.
constexpr size_t kBjDescBytes = 128;
size_t block_jacobi_bytes(int m);
int block_jacobi(const std::vector<JacobiJob>& jobs, const JacobiJob* jobs_dev, char* work,
                 void* dv_dev, double* norms_dev, int max_sweeps, double tol, hipStream_t st);

// Hermitian eigensolver dispatch: matrices up to kSmallJacobi on one
// workgroup each, larger ones by block Jacobi.
constexpr int kSmallJacobi = 256;
struct EigWork {
  char* bj = nullptr;       // block Jacobi buffers
  void* dv = nullptr;       // descriptors
  double* norms = nullptr;  // per-job norms
};
size_t eig_work_bytes(const std::vector<int>& ms);
void carve_eig_work(struct Arena& ar, const std::vector<int>& ms, EigWork& w);
int reduced_eig(std::vector<JacobiJob> jobs, JacobiJob* jobs_dev, const EigWork& w,
                int max_sweeps, double tol, hipStream_t st);
// 2-norms of the m columns of X (n x m, leading dimension ldx) into nrm (m
// doubles); the columns with nrm > thr * max(nrm) listed in idx (ascending)
// with scale = 1 / nrm, their number in *kept (all device memory)
int col_norm_keep(const c128* X, int64_t n, int64_t ldx, int m, double thr, double* nrm,
                  int32_t* idx, double* scale, int32_t* kept, hipStream_t st);
int gram_keep(const double* s, int m, double drop, int32_t* idx, double* scale, int32_t* kept,
              hipStream_t st);

}  // namespace fb
