// Work items of the batched solve and residual launches.
#pragma once
#include "fb_internal.h"

namespace fb {

// One tile of right-hand sides of one shifted system in one direction.
struct SolveJob {
  int32_t sys;    // factor set index
  int32_t dir;    // 0: A x = y, 1: A^H x = y
  int32_t col0;   // first column of the tile
  int32_t ncol;   // columns in the tile (<= tile width)
  const c128* in; // right-hand sides (columns from col0)
  c128* mid;      // forward-sweep intermediates (may alias in or out)
  c128* out;      // solution (written, or added to when add != 0)
  int64_t ldin, ldmid, ldout;
  int32_t add;
  int32_t pad_;
};

// r = y - A x for one tile (A = zI - B, or its conjugate transpose).
struct ResJob {
  const c128* x;
  const c128* y;
  c128* r;
  int64_t ldx, ldy, ldr;
  int32_t col0, ncol, dir, pad_;
  c128 z;
};

template <typename R>
int launch_solve_jobs(const cx<R>* mats, const int16_t* perm, int64_t n, int b, int njobs,
                      const SolveJob* jobs_dev, hipStream_t st);
template <typename R>
int launch_lu_impl(const Band& bd, int nsys, const c128* z_dev, cx<R>* mats, int16_t* perm,
                   int32_t* info, cx<R>* scratch, hipStream_t st);
template <typename R>
size_t lu_window_scratch(int b, int nsys);

template <typename R>
int solve_tile(int b);

size_t residual_part_doubles(int64_t n, int njobs);
int launch_residual_jobs(const Band& bd, int njobs, const ResJob* jobs_dev, double* part,
                         double* ratio_dev, hipStream_t st);

}  // namespace fb
