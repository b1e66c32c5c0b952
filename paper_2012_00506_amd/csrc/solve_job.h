// Work items of the batched solve and residual launches.
#pragma once
#include <algorithm>
#include <vector>
#include "fb_internal.h"

namespace fb {

// One tile of right-hand sides of one shifted system in one direction.
struct SolveJob {
  int32_t sys;    // factor set index
  int32_t dir;    // 0: A x = y, 1: A^H x = y
  int32_t col0;   // first column of the tile
  int32_t ncol;   // columns in the tile (<= tile width)
  const c128* in; // right-hand sides (columns from col0)
  void* mid;      // forward-sweep intermediates in the factors' complex type,
                  // ldmid in those elements; may alias in or out column by
                  // column (same column start, ldmid = ld * 16 / element size)
  c128* out;      // solution (written, or added to when add != 0)
  int64_t ldin, ldmid, ldout;
  int32_t add;
  int32_t grp;    // residual group of a correction job (the launch's gate array
                  // says whether it still runs)
};

// r = y - A x for one tile (A = zI - B, or its conjugate transpose).
struct ResJob {
  const c128* x;
  const c128* y;
  c128* r;
  int64_t ldx, ldy, ldr;
  int32_t col0, ncol, dir, grp;  // grp: index of the group in the call
  c128 z;
};

// Block size of the factor blocks: the band rounded up to the 16-row MFMA tile.
inline int block_size(int b) { return (b + 15) / 16 * 16; }

// mats: the factor blocks; matsT: their transposed copy, read by the
// conjugate-transposed solves (required for complex64, null for complex128)
// gate (dev, may be null): a job runs only while gate[job.grp] != 0
template <typename R>
int launch_solve_jobs(const cx<R>* mats, const cx<R>* matsT, const int16_t* perm, int64_t n,
                      int b, int njobs, const SolveJob* jobs_dev, double work, hipStream_t st,
                      const int32_t* gate = nullptr);
template <typename R>
int launch_lu_impl(const Band& bd, int nsys, const c128* z_dev, cx<R>* mats, cx<R>* matsT,
                   int16_t* perm, int32_t* info, cx<R>* scratch, cx<R>* lscr, hipStream_t st);
template <typename R>
size_t lu_window_scratch(int b, int nsys);

template <typename R>
int solve_tile(int b);

size_t residual_part_doubles(int64_t n, int njobs);
// columns per residual job for block size nb
int residual_cols(int nb);
// Residual of every job (group) whose gate entry is set (all when gate is
// null), then the refinement decision per group: ratio[g] = max over its
// columns of ||r|| / ||y||; flag[g] = 1 when the group needs a correction
// pass (ir, ratio above ir_tol, pass < max_pass and, after pass 0, the last
// pass at least halved the ratio); npass[g] counts the passes asked for.
struct RefineCtl {
  const int32_t* gate;  // null in pass 0
  int32_t* flag;
  double* ratio;
  int32_t* npass;
  int pass, max_pass, ir;
  double ir_tol;
};
int launch_residual_jobs(const Band& bd, int njobs, const ResJob* jobs_dev, double* part,
                         const RefineCtl& ctl, double work, hipStream_t st);
// algorithmic flops: solve 24 n b per column (L: n b, U: 2 n b complex MACs),
// FP64 residual 8 (2b+1) n per column
inline double solve_flops(int64_t n, int b, double cols) { return 24.0 * (double)n * b * cols; }
inline double resid_flops(int64_t n, int b, double cols) {
  return 8.0 * (2.0 * b + 1.0) * (double)n * cols;
}

// Shifted-system factors of one call.
template <typename R>
struct FactorBufs {
  cx<R>* mats = nullptr;
  cx<R>* matsT = nullptr;  // complex64: every block transposed (H solves)
  int16_t* perm = nullptr;
  int32_t* info = nullptr;
  cx<R>* scratch = nullptr;
  cx<R>* lscr = nullptr;  // per system 2 x 2nb x nb multiplier scratch
  c128* z = nullptr;
};
template <typename R>
void carve_factors(Arena& ar, const Band& bd, int nsys, FactorBufs<R>& f);
// z_host: 2*nsys doubles (re, im); returns FB_ERR_SINGULAR on a zero pivot
template <typename R>
int factor_systems(const Band& bd, int nsys, const double* z_host, FactorBufs<R>& f,
                   hipStream_t st);
// FB_ERR_SINGULAR when a factorisation met an exactly zero pivot (synchronises)
template <typename R>
int factor_check(int nsys, FactorBufs<R>& f, hipStream_t st);

// Buffers of the solve + refinement driver.
struct RefineBufs {
  int tile = 32;
  int gcols = 32;  // columns per residual group
  int cap_jobs = 0;
  size_t wave = 0;           // groups whose residual blocks fit at once
  SolveJob* jobs_dev = nullptr;
  ResJob* rjobs_dev = nullptr;   // one per group (cap_jobs)
  SolveJob* cjobs_dev = nullptr; // correction jobs of every group
  c128* rbuf = nullptr;          // residual blocks of one wave of groups
  double* part = nullptr;
  double* ratio = nullptr;       // per group
  int32_t* flag = nullptr;       // per group
  int32_t* npass = nullptr;      // per group
};
void carve_refine(Arena& ar, const Band& bd, int tile, int max_jobs, bool ir, bool need_res,
                  RefineBufs& rb);

// Complex128 fallback of the refined complex64 solves: a system whose FP64
// residual stays above ir_tol after ir_max correction passes is factored
// again in complex128 (cap systems at a time, in f) and its columns are
// solved again from the right-hand sides; its sys_pass entry becomes -1.
struct C128Fallback {
  FactorBufs<double>* f = nullptr;
  int cap = 0;
  // the system held in each slot of f, kept between calls with the same
  // shifts (FEAST iterations of one wave); whoever changes the shifts of the
  // system indices calls reset()
  mutable std::vector<int> slot_sys;
  // systems that fell back in an earlier call with the same shifts: later
  // calls solve them in complex128 at once
  mutable std::vector<int> known;
  void reset() const {
    slot_sys.clear();
    known.clear();
  }
};
// systems the fallback factors hold at once: two for one-off solves, a
// quarter of a FEAST wave's systems, whose factors are kept between iterations
inline int fallback_cap(int nsys) { return nsys < 2 ? nsys : 2; }
inline int feast_fallback_cap(int nsys) { return std::min(nsys, std::max(2, nsys / 4)); }
size_t refine_bytes(const Band& bd, int tile, int max_jobs, bool ir, bool need_res);
// Solve + refinement of one batch of jobs in three stages (solve_refine runs
// all three): tables to the device, kernel launches (no host round-trip, so
// they can be captured), read-back and complex128 fallback.
struct RefinePlan {
  int njobs = 0, ng = 0, maxpass = 0;
  bool ir = false, need_res = false;
  double ir_tol = 0.0, cols = 0.0;
  std::vector<std::pair<int, int>> groups;
  std::vector<double> gcols;
  std::vector<size_t> cj_off;
};
template <typename R>
int refine_prepare(const Band& bd, const std::vector<SolveJob>& jobs,
                   const std::vector<c128>& zsys, bool ir, double ir_tol, int ir_max,
                   bool need_res, RefineBufs& rb, RefinePlan& plan, hipStream_t st);
template <typename R>
int refine_launch(const Band& bd, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                  const RefinePlan& plan, RefineBufs& rb, hipStream_t st);
// stagnated (may be null): systems that ended above ir_tol before any fallback
template <typename R>
int refine_finish(const Band& bd, const std::vector<SolveJob>& jobs,
                  const std::vector<c128>& zsys, const RefinePlan& plan, RefineBufs& rb,
                  std::vector<double>& sys_res, std::vector<int32_t>& sys_pass, int* unconverged,
                  hipStream_t st, const C128Fallback* fb, int* stagnated);
template <typename R>
int solve_refine(const Band& bd, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                 const std::vector<SolveJob>& jobs, const std::vector<c128>& zsys, bool ir,
                 double ir_tol, int ir_max, bool need_res, RefineBufs& rb,
                 std::vector<double>& sys_res, std::vector<int32_t>& sys_pass, int* unconverged,
                 hipStream_t st, const C128Fallback* fb = nullptr);
int check_band(const fb_band* B);

}  // namespace fb
