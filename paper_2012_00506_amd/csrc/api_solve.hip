// C ABI: band_inertia, band_shifted_solve, fb_strerror, fb_device_info.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "solve_job.h"
#include "prof.h"

namespace fb {

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

int check_band(const fb_band* B) {
  if (!B) return -1;
  if (B->n < 1 || B->b < 0 || B->b >= B->n) return -1;
  if (B->dtype != FB_REAL64 && B->dtype != FB_COMPLEX128) return -1;
  if (B->ldab < B->b + 1 || B->ab == nullptr) return -1;
  if (B->b > 128) return -1;  // block kernels are sized for b <= 128
  return 0;
}

template <typename R>
void carve_factors(Arena& ar, const Band& bd, int nsys, FactorBufs<R>& f) {
  const int nb = block_size(bd.b);
  int K = (int)((bd.n + nb - 1) / nb);
  size_t bb = (size_t)nb * nb;
  f.mats = ar.take<cx<R>>((size_t)nsys * K * 5 * bb);
  f.matsT = sizeof(R) == 4 ? ar.take<cx<R>>((size_t)nsys * K * 5 * bb) : nullptr;
  f.perm = ar.take<int16_t>((size_t)nsys * K * 2 * nb);
  f.info = ar.take<int32_t>(nsys);
  size_t sc = lu_window_scratch<R>(bd.b, nsys);
  f.scratch = sc ? ar.take<cx<R>>(sc / sizeof(cx<R>)) : nullptr;
  f.lscr = ar.take<cx<R>>((size_t)nsys * 4 * bb);
  f.z = ar.take<c128>(nsys);
}

template <typename R>
int factor_systems(const Band& bd, int nsys, const double* z_host, FactorBufs<R>& f,
                   hipStream_t st) {
  FB_HIP(hipMemcpyAsync(f.z, z_host, sizeof(c128) * nsys, hipMemcpyHostToDevice, st));
  FB_TRY(launch_lu_impl<R>(bd, nsys, f.z, f.mats, f.matsT, f.perm, f.info, f.scratch, f.lscr,
                           st));
  std::vector<int32_t> info(nsys);
  FB_HIP(hipMemcpyAsync(info.data(), f.info, sizeof(int32_t) * nsys, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  for (int s = 0; s < nsys; ++s)
    if (info[s] != 0) return FB_ERR_SINGULAR;
  return 0;
}


template <typename R>
int factor_check(int nsys, FactorBufs<R>& f, hipStream_t st) {
  std::vector<int32_t> info(nsys);
  FB_HIP(hipMemcpyAsync(info.data(), f.info, sizeof(int32_t) * nsys, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  for (int s = 0; s < nsys; ++s)
    if (info[s] != 0) return FB_ERR_SINGULAR;
  return 0;
}

template int factor_check<float>(int, FactorBufs<float>&, hipStream_t);
template int factor_check<double>(int, FactorBufs<double>&, hipStream_t);
template void carve_factors<float>(Arena&, const Band&, int, FactorBufs<float>&);
template void carve_factors<double>(Arena&, const Band&, int, FactorBufs<double>&);
template int factor_systems<float>(const Band&, int, const double*, FactorBufs<float>&, hipStream_t);
template int factor_systems<double>(const Band&, int, const double*, FactorBufs<double>&, hipStream_t);

}  // namespace fb

using namespace fb;

extern "C" const char* fb_strerror(int code) {
  switch (code) {
    case 0: return "success";
    case FB_ERR_SINGULAR: return "a shifted system has an exactly zero pivot";
    case FB_ERR_NOT_BUILT: return "no kernel for this device";
    case FB_ERR_CERTIFY: return "a slice boundary could not be certified";
    case FB_ERR_NOMEM: return "workspace too small";
    case FB_ERR_NONFINITE: return "NaN or Inf in an input block";
    case FB_ERR_INTERNAL: return "internal error";
    case FB_ERR_TOO_LARGE: return "the problem exceeds the fixed scratch of the no-allocation entry point";
    default: break;
  }
  if (code <= -1000 && code > -2000) return hipGetErrorString((hipError_t)(-1000 - code));
  if (code < 0 && code > -100) return "invalid argument";
  if (code > 0) return "some slices or systems did not converge";
  return "unknown error";
}

extern "C" int fb_device_info(int32_t* cus, char* name, int32_t cap) {
  int dev = 0;
  FB_HIP(hipGetDevice(&dev));
  hipDeviceProp_t p;
  FB_HIP(hipGetDeviceProperties(&p, dev));
  if (cus) *cus = p.multiProcessorCount;
  if (name && cap > 0) {
    strncpy(name, p.gcnArchName, (size_t)cap - 1);
    name[cap - 1] = 0;
  }
  return 0;
}

extern "C" int band_inertia(const fb_band* B, int32_t nshift, const double* shifts,
                            int32_t* n_neg, int32_t* n_zero, int32_t* n_pos, void* work,
                            size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (nshift < 0) return -2;
  if (nshift > 0 && !shifts) return -3;
  if (nshift > 0 && !n_neg) return -4;
  if (!lwork) return -8;
  hipStream_t st = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st, false));
  double* sh = ar.take<double>(std::max(nshift, 1));
  int32_t* cnt = ar.take<int32_t>(3 * (size_t)std::max(nshift, 1));
  size_t scb = inertia_scratch_bytes(bd, nshift);
  void* scratch = scb ? (void*)ar.take<char>(scb) : nullptr;
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  if (nshift == 0) return 0;
  for (int i = 0; i < nshift; ++i)
    if (!isfinite(shifts[i])) return -3;
  FB_HIP(hipMemcpyAsync(sh, shifts, sizeof(double) * nshift, hipMemcpyHostToDevice, st));
  FB_TRY(launch_inertia(bd, nshift, sh, cnt, scratch, st));
  std::vector<int32_t> h(3 * (size_t)nshift);
  FB_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * 3 * nshift, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nshift; ++i) {
    n_neg[i] = h[3 * i];
    if (n_zero) n_zero[i] = h[3 * i + 1];
    if (n_pos) n_pos[i] = h[3 * i + 2];
  }
  return 0;
}

namespace fb {

// Largest number of tiles refined together (bounds the residual buffers).
size_t ir_wave_jobs(int64_t n, int tile) {
  const size_t cap = (size_t)8 << 30;
  size_t per = (size_t)n * tile * sizeof(c128);
  size_t w = cap / per;
  return std::max<size_t>(w, 64);
}

void carve_refine(Arena& ar, const Band& bd, int tile, int max_jobs, bool ir, bool need_res,
                  RefineBufs& rb) {
  rb.tile = tile;
  rb.gcols = residual_cols(block_size(bd.b));  // >= tile (variant_fits)
  rb.cap_jobs = std::max(max_jobs, 1);
  rb.jobs_dev = ar.take<SolveJob>(rb.cap_jobs);
  rb.wave = need_res ? std::min<size_t>(ir_wave_jobs(bd.n, rb.gcols), (size_t)rb.cap_jobs) : 0;
  // every group has a residual job; a group's corrections are its tiles
  rb.rjobs_dev = need_res ? ar.take<ResJob>(rb.cap_jobs) : nullptr;
  rb.cjobs_dev = ir ? ar.take<SolveJob>(rb.cap_jobs) : nullptr;
  rb.rbuf = need_res ? ar.take<c128>(rb.wave * (size_t)bd.n * rb.gcols) : nullptr;
  rb.part = need_res ? ar.take<double>(residual_part_doubles(bd.n, (int)rb.wave)) : nullptr;
  rb.ratio = need_res ? ar.take<double>(rb.cap_jobs) : nullptr;
  rb.flag = need_res ? ar.take<int32_t>(rb.cap_jobs) : nullptr;
  rb.npass = need_res ? ar.take<int32_t>(rb.cap_jobs) : nullptr;
}

size_t refine_bytes(const Band& bd, int tile, int max_jobs, bool ir, bool need_res) {
  Arena q;
  RefineBufs rb;
  carve_refine(q, bd, tile, max_jobs, ir, need_res, rb);
  return q.used;
}

// The solve jobs, then (need_res) the FP64 residual ||y - A x|| / ||y|| per
// group of adjacent tiles (same system, direction and blocks, up to gcols
// columns) and (ir) correction solves of the groups above ir_tol.  The
// decisions are taken on the device: each residual launch sets a flag per
// group that gates the next correction and residual launches (a group stops
// when it meets ir_tol, after ir_max passes, or when a pass did not halve its
// residual), so the launches of a call run without host round-trips and can
// be captured in a graph; the ratios are read back once at the end.  Groups
// are processed in waves that bound the residual buffers.
//   refine_prepare: job tables to the device (before any capture)
//   refine_launch:  every kernel launch of the call (capturable)
//   refine_finish:  ratios read back, complex128 fallback of stagnated systems
template <typename R>
int refine_prepare(const Band& bd, const std::vector<SolveJob>& jobs,
                   const std::vector<c128>& zsys, bool ir, double ir_tol, int ir_max,
                   bool need_res, RefineBufs& rb, RefinePlan& plan, hipStream_t st) {
  plan = RefinePlan{};
  const int njobs = (int)jobs.size();
  plan.njobs = njobs;
  plan.ir = ir;
  plan.need_res = need_res;
  plan.ir_tol = ir_tol;
  plan.maxpass = ir ? ir_max : 0;
  if (njobs == 0) return 0;
  if (njobs > rb.cap_jobs) return FB_ERR_INTERNAL;
  FB_HIP(hipMemcpyAsync(rb.jobs_dev, jobs.data(), sizeof(SolveJob) * njobs, hipMemcpyHostToDevice, st));
  for (const SolveJob& jb : jobs) plan.cols += jb.ncol;
  if (!need_res) return 0;
  // groups [first, last] of consecutive jobs
  auto& groups = plan.groups;
  for (int i = 0; i < njobs; ++i) {
    if (!groups.empty()) {
      const SolveJob& f = jobs[groups.back().first];
      const SolveJob& p = jobs[groups.back().second];
      const SolveJob& c = jobs[i];
      if (c.sys == p.sys && c.dir == p.dir && c.in == p.in && c.out == p.out &&
          c.ldin == p.ldin && c.ldout == p.ldout && c.col0 == p.col0 + p.ncol &&
          c.col0 + c.ncol - f.col0 <= rb.gcols) {
        groups.back().second = i;
        continue;
      }
    }
    groups.push_back({i, i});
  }
  const int ng = (int)groups.size();
  plan.ng = ng;
  // residual job of every group (its block in the wave's residual buffer)
  // and the correction jobs of every group, contiguous per wave
  std::vector<ResJob> rj(ng);
  std::vector<SolveJob> cj;
  plan.gcols.assign(ng, 0.0);
  for (int g = 0; g < ng; ++g) {
    if ((size_t)g % rb.wave == 0) plan.cj_off.push_back(cj.size());
    const SolveJob& f = jobs[groups[g].first];
    const SolveJob& l = jobs[groups[g].second];
    ResJob& r = rj[g];
    r.x = f.out;
    r.y = f.in;
    r.r = rb.rbuf + ((size_t)g % rb.wave) * (size_t)bd.n * rb.gcols - (int64_t)f.col0 * bd.n;
    r.ldx = f.ldout;
    r.ldy = f.ldin;
    r.ldr = bd.n;
    r.col0 = f.col0;
    r.ncol = l.col0 + l.ncol - f.col0;
    r.dir = f.dir;
    r.grp = g;
    r.z = zsys[f.sys];
    plan.gcols[g] = r.ncol;
    if (ir)
      for (int i = groups[g].first; i <= groups[g].second; ++i) {
        SolveJob c = jobs[i];
        c.in = r.r;
        c.mid = r.r;
        c.ldin = bd.n;
        c.ldmid = bd.n * (int64_t)(sizeof(c128) / sizeof(cx<R>));
        c.add = 1;
        c.grp = g;
        cj.push_back(c);
      }
  }
  plan.cj_off.push_back(cj.size());
  if (cj.size() > (size_t)rb.cap_jobs) return FB_ERR_INTERNAL;
  FB_HIP(hipMemcpyAsync(rb.rjobs_dev, rj.data(), sizeof(ResJob) * ng, hipMemcpyHostToDevice, st));
  if (ir && !cj.empty())
    FB_HIP(hipMemcpyAsync(rb.cjobs_dev, cj.data(), sizeof(SolveJob) * cj.size(),
                          hipMemcpyHostToDevice, st));
  return 0;
}

template <typename R>
int refine_launch(const Band& bd, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                  const RefinePlan& plan, RefineBufs& rb, hipStream_t st) {
  if (plan.njobs == 0) return 0;
  FB_TRY(launch_solve_jobs<R>(mats, matsT, perm, bd.n, bd.b, plan.njobs, rb.jobs_dev,
                              solve_flops(bd.n, bd.b, plan.cols), st));
  if (!plan.need_res) return 0;
  for (size_t w0 = 0, wi = 0; w0 < (size_t)plan.ng; w0 += rb.wave, ++wi) {
    const int nw = (int)std::min(rb.wave, (size_t)plan.ng - w0);
    double wcols = 0;
    for (int g = 0; g < nw; ++g) wcols += plan.gcols[w0 + g];
    RefineCtl ctl{nullptr, rb.flag, rb.ratio, rb.npass, 0, plan.maxpass, plan.ir ? 1 : 0,
                  plan.ir_tol};
    FB_TRY(launch_residual_jobs(bd, nw, rb.rjobs_dev + w0, rb.part, ctl,
                                resid_flops(bd.n, bd.b, wcols), st));
    for (int pass = 1; pass <= plan.maxpass; ++pass) {
      // gated launches: their work is added once the passes are known
      FB_TRY(launch_solve_jobs<R>(mats, matsT, perm, bd.n, bd.b,
                                  (int)(plan.cj_off[wi + 1] - plan.cj_off[wi]),
                                  rb.cjobs_dev + plan.cj_off[wi], 0.0, st, rb.flag));
      ctl.gate = rb.flag;
      ctl.pass = pass;
      FB_TRY(launch_residual_jobs(bd, nw, rb.rjobs_dev + w0, rb.part, ctl, 0.0, st));
    }
  }
  return 0;
}

// Columns of the given systems solved anew from the right-hand sides in
// complex128 with the fallback factors (jobs of other systems are ignored):
// sys_res gets their FP64 residual ratios, sys_pass -1.
static int fallback_solve(const Band& bd, const std::vector<SolveJob>& jobs,
                          const std::vector<int>& systems, const std::vector<c128>& zsys,
                          RefineBufs& rb, std::vector<double>& sys_res,
                          std::vector<int32_t>& sys_pass, hipStream_t st, const C128Fallback* fb) {
  // factors kept from earlier calls are reused; the missing systems are
  // factored (one launch) into the free slots, and all slots start over when
  // they do not fit
  const int nbk = block_size(bd.b);
  const int K = (int)((bd.n + nbk - 1) / nbk);
  std::vector<int>& ss = fb->slot_sys;
  std::vector<int> todo = systems;
  while (!todo.empty()) {
    std::vector<int> missing;
    for (int s : todo)
      if (std::find(ss.begin(), ss.end(), s) == ss.end()) missing.push_back(s);
    if (ss.size() + missing.size() > (size_t)fb->cap) {
      ss.clear();
      missing.assign(todo.begin(), todo.begin() + std::min(todo.size(), (size_t)fb->cap));
    }
    if (!missing.empty()) {
      const size_t at = ss.size();
      std::vector<double> zh(2 * missing.size());
      for (size_t q = 0; q < missing.size(); ++q) {
        zh[2 * q] = zsys[missing[q]].x;
        zh[2 * q + 1] = zsys[missing[q]].y;
      }
      FactorBufs<double> view = *fb->f;  // slots at .. at + missing - 1
      view.mats += at * K * 5 * (size_t)nbk * nbk;
      view.perm += at * K * 2 * (size_t)nbk;
      view.info += at;
      view.z += at;
      FB_TRY(factor_systems<double>(bd, (int)missing.size(), zh.data(), view, st));
      ss.insert(ss.end(), missing.begin(), missing.end());
    }
    std::vector<int> rest;
    std::vector<SolveJob> sub;
    for (int s : todo)
      if (std::find(ss.begin(), ss.end(), s) == ss.end()) rest.push_back(s);
    for (const SolveJob& jb : jobs) {
      if (std::find(todo.begin(), todo.end(), jb.sys) == todo.end()) continue;
      auto it = std::find(ss.begin(), ss.end(), jb.sys);
      if (it == ss.end()) continue;
      SolveJob c = jb;
      c.sys = (int32_t)(it - ss.begin());
      c.mid = c.out;
      c.ldmid = c.ldout;
      c.add = 0;
      sub.push_back(c);
    }
    std::vector<c128> zsub(ss.size());
    for (size_t q = 0; q < ss.size(); ++q) zsub[q] = zsys[ss[q]];
    std::vector<double> sres(ss.size(), 0.0);
    std::vector<int32_t> spass(ss.size(), 0);
    FB_TRY(solve_refine<double>(bd, fb->f->mats, nullptr, fb->f->perm, sub, zsub, false, 0.0, 0,
                                true, rb, sres, spass, nullptr, st));
    for (int s : todo) {
      auto it = std::find(ss.begin(), ss.end(), s);
      if (it == ss.end()) continue;
      sys_res[s] = sres[it - ss.begin()];
      sys_pass[s] = -1;
    }
    todo.swap(rest);
  }
  return 0;
}

template <typename R>
int refine_finish(const Band& bd, const std::vector<SolveJob>& jobs,
                  const std::vector<c128>& zsys, const RefinePlan& plan, RefineBufs& rb,
                  std::vector<double>& sys_res, std::vector<int32_t>& sys_pass, int* unconverged,
                  hipStream_t st, const C128Fallback* fb, int* stagnated) {
  if (plan.njobs == 0 || !plan.need_res) return 0;
  const int ng = plan.ng;
  const double ir_tol = plan.ir_tol;
  std::vector<double> ratio(ng);
  std::vector<int32_t> npass(ng);
  FB_HIP(hipMemcpyAsync(ratio.data(), rb.ratio, sizeof(double) * ng, hipMemcpyDeviceToHost, st));
  FB_HIP(hipMemcpyAsync(npass.data(), rb.npass, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, st));
  FB_HIP(hipStreamSynchronize(st));
  std::vector<int> failed;  // systems with a group above ir_tol at the end
  double corr_cols = 0;
  for (int g = 0; g < ng; ++g) {
    const int sys = jobs[plan.groups[g].first].sys;
    if (!(ratio[g] <= sys_res[sys])) sys_res[sys] = ratio[g];
    sys_pass[sys] = std::max(sys_pass[sys], npass[g]);
    corr_cols += (double)npass[g] * plan.gcols[g];
    if (plan.ir && !(ratio[g] <= ir_tol)) failed.push_back(sys);
  }
  prof_add_work(FB_PROF_SOLVE, solve_flops(bd.n, bd.b, corr_cols));
  prof_add_work(FB_PROF_RESID, resid_flops(bd.n, bd.b, corr_cols));
  if (stagnated) *stagnated = (int)failed.size();
  std::sort(failed.begin(), failed.end());
  failed.erase(std::unique(failed.begin(), failed.end()), failed.end());
  if (!failed.empty() && fb && fb->f && fb->cap > 0 && sizeof(R) == 4) {
    FB_TRY(fallback_solve(bd, jobs, failed, zsys, rb, sys_res, sys_pass, st, fb));
    for (int s : failed)
      if (std::find(fb->known.begin(), fb->known.end(), s) == fb->known.end())
        fb->known.push_back(s);
  }
  if (unconverged)
    for (int s : failed)
      if (!(sys_res[s] <= ir_tol)) ++*unconverged;
  return 0;
}


template <typename R>
int solve_refine(const Band& bd, const cx<R>* mats, const cx<R>* matsT, const int16_t* perm,
                 const std::vector<SolveJob>& jobs, const std::vector<c128>& zsys, bool ir,
                 double ir_tol, int ir_max, bool need_res, RefineBufs& rb,
                 std::vector<double>& sys_res, std::vector<int32_t>& sys_pass, int* unconverged,
                 hipStream_t st, const C128Fallback* fb) {
  if (fb && fb->f && fb->cap > 0 && sizeof(R) == 4 && need_res && !fb->known.empty()) {
    // systems that fell back in an earlier call go to complex128 at once
    std::vector<SolveJob> keep;
    std::vector<int> direct;
    for (const SolveJob& jb : jobs) {
      if (std::find(fb->known.begin(), fb->known.end(), jb.sys) == fb->known.end()) {
        keep.push_back(jb);
      } else if (std::find(direct.begin(), direct.end(), jb.sys) == direct.end()) {
        direct.push_back(jb.sys);
      }
    }
    if (!direct.empty()) {
      FB_TRY(fallback_solve(bd, jobs, direct, zsys, rb, sys_res, sys_pass, st, fb));
      if (unconverged)
        for (int s : direct)
          if (!(sys_res[s] <= ir_tol)) ++*unconverged;
      RefinePlan plan;
      FB_TRY(refine_prepare<R>(bd, keep, zsys, ir, ir_tol, ir_max, need_res, rb, plan, st));
      FB_TRY(refine_launch<R>(bd, mats, matsT, perm, plan, rb, st));
      return refine_finish<R>(bd, keep, zsys, plan, rb, sys_res, sys_pass, unconverged, st, fb,
                              nullptr);
    }
  }
  RefinePlan plan;
  FB_TRY(refine_prepare<R>(bd, jobs, zsys, ir, ir_tol, ir_max, need_res, rb, plan, st));
  FB_TRY(refine_launch<R>(bd, mats, matsT, perm, plan, rb, st));
  return refine_finish<R>(bd, jobs, zsys, plan, rb, sys_res, sys_pass, unconverged, st, fb,
                          nullptr);
}

#define FB_REFINE_INST(R)                                                                      \
  template int refine_prepare<R>(const Band&, const std::vector<SolveJob>&,                    \
                                 const std::vector<c128>&, bool, double, int, bool,            \
                                 RefineBufs&, RefinePlan&, hipStream_t);                       \
  template int refine_launch<R>(const Band&, const cx<R>*, const cx<R>*, const int16_t*,       \
                                const RefinePlan&, RefineBufs&, hipStream_t);                  \
  template int refine_finish<R>(const Band&, const std::vector<SolveJob>&,                     \
                                const std::vector<c128>&, const RefinePlan&, RefineBufs&,      \
                                std::vector<double>&, std::vector<int32_t>&, int*, hipStream_t, \
                                const C128Fallback*, int*);
FB_REFINE_INST(float)
FB_REFINE_INST(double)
#undef FB_REFINE_INST

template int solve_refine<float>(const Band&, const c64*, const c64*, const int16_t*,
                                 const std::vector<SolveJob>&, const std::vector<c128>&, bool,
                                 double, int, bool, RefineBufs&, std::vector<double>&,
                                 std::vector<int32_t>&, int*, hipStream_t, const C128Fallback*);
template int solve_refine<double>(const Band&, const c128*, const c128*, const int16_t*,
                                  const std::vector<SolveJob>&, const std::vector<c128>&, bool,
                                  double, int, bool, RefineBufs&, std::vector<double>&,
                                  std::vector<int32_t>&, int*, hipStream_t, const C128Fallback*);

template <typename R>
int shifted_solve_impl(const fb_band* B, int nsys, const double* z, const int32_t* m,
                       const void* const* Y, const int64_t* ldy, void* const* X,
                       void* const* XH, const int64_t* ldx, double* resid, int32_t* passes,
                       const fb_solve_opts* o, void* work, size_t* lwork, hipStream_t st) {
  const bool ir = (o->precision == 1);
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  double* fpart = ar.take<double>((size_t)kFiniteParts * std::max(nsys, 1));
  FactorBufs<R> f;
  carve_factors<R>(ar, bd, nsys, f);
  FactorBufs<double> f64fb;
  C128Fallback fbk;
  if (ir) {
    fbk.cap = fallback_cap(nsys);
    carve_factors<double>(ar, bd, fbk.cap, f64fb);
    fbk.f = &f64fb;
  }

  // jobs: every (system, direction, tile)
  const int tile = solve_tile<R>(bd.b);
  std::vector<SolveJob> jobs;
  for (int s = 0; s < nsys; ++s)
    for (int dir = 0; dir < 2; ++dir) {
      c128* out = (c128*)(dir == 0 ? X[s] : (XH ? XH[s] : nullptr));
      if (!out) continue;
      for (int c0 = 0; c0 < m[s]; c0 += tile) {
        SolveJob jb{};
        jb.sys = s;
        jb.dir = dir;
        jb.col0 = c0;
        jb.ncol = std::min(tile, m[s] - c0);
        jb.in = (const c128*)Y[s];
        jb.mid = out;
        jb.out = out;
        jb.ldin = ldy[s];
        jb.ldmid = ldx[s] * (int64_t)(sizeof(c128) / sizeof(cx<R>));
        jb.ldout = ldx[s];
        jobs.push_back(jb);
      }
    }
  const bool need_res = ir || resid != nullptr;
  RefineBufs rb;
  carve_refine(ar, bd, tile, (int)jobs.size(), ir, need_res, rb);
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  FB_TRY(check_finite_blocks(nsys, Y, ldy, m, bd.n, true, fpart, st));

  FB_TRY(factor_systems<R>(bd, nsys, z, f, st));
  std::vector<c128> zsys(nsys);
  for (int s = 0; s < nsys; ++s) zsys[s] = mk(z[2 * s], z[2 * s + 1]);
  std::vector<double> sys_res(nsys, 0.0);
  std::vector<int32_t> sys_pass(nsys, 0);
  int unconverged = 0;
  FB_TRY(solve_refine<R>(bd, f.mats, f.matsT, f.perm, jobs, zsys, ir, o->ir_tol, o->ir_max, need_res, rb,
                         sys_res, sys_pass, &unconverged, st, ir ? &fbk : nullptr));
  FB_HIP(hipStreamSynchronize(st));
  if (resid)
    for (int s = 0; s < nsys; ++s) resid[s] = sys_res[s];
  if (passes)
    for (int s = 0; s < nsys; ++s) passes[s] = sys_pass[s];
  if (unconverged) {
    int ns = 0;
    for (int s = 0; s < nsys; ++s) ns += (ir && sys_res[s] > o->ir_tol) ? 1 : 0;
    return ns;
  }
  return 0;
}

}  // namespace fb

extern "C" int band_shifted_solve(const fb_band* B, int32_t nsys, const double* z,
                                  const int32_t* m, const void* const* Y, const int64_t* ldy,
                                  void* const* X, void* const* XH, const int64_t* ldx,
                                  double* resid, int32_t* passes, const fb_solve_opts* o,
                                  void* work, size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (nsys < 0) return -2;
  if (nsys > 0 && !z) return -3;
  if (nsys > 0 && !m) return -4;
  if (nsys > 0 && (!Y || !ldy)) return -5;
  if (nsys > 0 && !X) return -7;
  if (nsys > 0 && !ldx) return -9;
  if (!o) return -12;
  if (!lwork) return -14;
  if (o->precision != 0 && o->precision != 1) return -12;
  if (o->precision == 1 && (!(o->ir_tol > 0) || o->ir_max < 0)) return -12;
  for (int s = 0; s < nsys; ++s) {
    if (m[s] < 0) return -4;
    if (!isfinite(z[2 * s]) || !isfinite(z[2 * s + 1])) return -3;
    if (m[s] > 0 && (!Y[s] || ldy[s] < B->n)) return -5;
    if (m[s] > 0 && (!X[s] || ldx[s] < B->n)) return -7;
  }
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == 1)
    return shifted_solve_impl<float>(B, nsys, z, m, Y, ldy, X, XH, ldx, resid, passes, o, work,
                                     lwork, st);
  return shifted_solve_impl<double>(B, nsys, z, m, Y, ldy, X, XH, ldx, resid, passes, o, work,
                                    lwork, st);
}
