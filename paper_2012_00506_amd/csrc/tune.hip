// Autotuner of the block-solve kernel: times every variant that fits in LDS
// on the caller's shape with HIP events and keeps the fastest per
// (precision, block size) for the rest of the process; results can be
// appended to and reloaded from a JSON-lines cache file.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "rr.h"
#include "solve_job.h"
#include "tune.h"

namespace fb {

namespace {
std::mutex g_mu;
std::map<std::pair<int, int>, int>& table() {
  static std::map<std::pair<int, int>, int> t;
  return t;
}
}  // namespace

bool variant_fits(size_t rsize, int nb, int v) {
  // a refinement residual group (residual_cols(nb) columns) must cover a tile
  if (variant_tile(v) > residual_cols(nb)) return false;
  const size_t lds = solve_lds_bytes(nb, variant_tile(v), 2 * rsize);
  return lds <= 160 * 1024;
}

int tuned_variant(size_t rsize, int nb) {
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = table().find({(int)rsize, nb});
    if (it != table().end() && variant_fits(rsize, nb, it->second)) return it->second;
  }
  // untuned default: 32-wide tiles; prefetch where the registers allow it
  int v = rsize == 4 ? 3 : 2;
  while (v > 0 && !variant_fits(rsize, nb, v)) v -= 2;
  return v;
}

void set_tuned_variant(size_t rsize, int nb, int v) {
  std::lock_guard<std::mutex> g(g_mu);
  table()[{(int)rsize, nb}] = v;
}

template <typename R>
int autotune_impl(const fb_band* B, int nsys, int m, const char* path, int32_t* chosen,
                  double* ms_out, void* work, size_t* lwork, hipStream_t st) {
  Arena ar;
  ar.base = (char*)work;
  ar.cap = *lwork;
  Band bd;
  FB_TRY(ingest_band(B, bd, ar, st));
  const int nb = block_size(bd.b);
  FactorBufs<R> f;
  carve_factors<R>(ar, bd, nsys, f);
  c128* Y = ar.take<c128>((size_t)bd.n * m);
  c128* X = ar.take<c128>((size_t)bd.n * m * nsys * 2);
  const int max_jobs = nsys * 2 * ((m + 15) / 16);
  SolveJob* jobs_dev = ar.take<SolveJob>(max_jobs);
  if (work == nullptr) {
    *lwork = ar.used;
    return 0;
  }
  if (!ar.fits()) return FB_ERR_NOMEM;
  double stats[3];
  FB_TRY(band_stats_host(bd, stats, st));
  std::vector<double> z(2 * nsys);
  for (int s = 0; s < nsys; ++s) {  // shifts spread over the Gershgorin interval
    z[2 * s] = stats[1] + (stats[2] - stats[1]) * (s + 0.5) / nsys;
    z[2 * s + 1] = 0.05 * (stats[2] - stats[1]) / nsys + 1e-3;
  }
  FB_TRY(factor_systems<R>(bd, nsys, z.data(), f, st));
  FB_TRY(fill_zero(Y, bd.n, m, bd.n, st));
  hipEvent_t e0, e1;
  FB_HIP(hipEventCreate(&e0));
  FB_HIP(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.f;
  std::vector<std::pair<int, float>> timed;
  for (int v = 0; v < kNumVariants; ++v) {
    if (!variant_fits(sizeof(R), nb, v)) continue;
    const int tile = variant_tile(v);
    std::vector<SolveJob> jobs;
    for (int s = 0; s < nsys; ++s)
      for (int dir = 0; dir < 2; ++dir)
        for (int c0 = 0; c0 < m; c0 += tile) {
          SolveJob jb{};
          jb.sys = s;
          jb.dir = dir;
          jb.col0 = c0;
          jb.ncol = std::min(tile, m - c0);
          jb.in = Y;
          jb.ldin = bd.n;
          jb.out = X + ((size_t)s * 2 + dir) * bd.n * m;
          jb.mid = jb.out;
          jb.ldout = bd.n;
          jb.ldmid = bd.n * (int64_t)(sizeof(c128) / sizeof(cx<R>));
          jobs.push_back(jb);
        }
    FB_HIP(hipMemcpyAsync(jobs_dev, jobs.data(), sizeof(SolveJob) * jobs.size(),
                          hipMemcpyHostToDevice, st));
    set_tuned_variant(sizeof(R), nb, v);
    FB_TRY(launch_solve_jobs<R>(f.mats, f.matsT, f.perm, bd.n, bd.b, (int)jobs.size(), jobs_dev, 0.0, st));
    FB_HIP(hipEventRecord(e0, st));
    for (int rep = 0; rep < 2; ++rep)
      FB_TRY(launch_solve_jobs<R>(f.mats, f.matsT, f.perm, bd.n, bd.b, (int)jobs.size(), jobs_dev, 0.0,
                                  st));
    FB_HIP(hipEventRecord(e1, st));
    FB_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FB_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms *= 0.5f;
    timed.push_back({v, ms});
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // The streamed variants hold one wave per SIMD: on a launch with fewer
  // workgroups than this full-batch problem (one slice at a time) they hide
  // less latency, so one wins only by a clear margin over the best of the rest.
  int best_s = -1;
  float best_s_ms = 0.f;
  for (const auto& tv : timed) {
    int& b = variant_streamed(tv.first) ? best_s : best;
    float& b_ms = variant_streamed(tv.first) ? best_s_ms : best_ms;
    if (b < 0 || tv.second < b_ms) {
      b = tv.first;
      b_ms = tv.second;
    }
  }
  if (best_s >= 0 && (best < 0 || best_s_ms < kStreamedMargin * best_ms)) {
    best = best_s;
    best_ms = best_s_ms;
  }
  if (best < 0) return FB_ERR_INTERNAL;
  set_tuned_variant(sizeof(R), nb, best);
  if (chosen) *chosen = best;
  if (ms_out) *ms_out = best_ms;
  if (path) {
    FILE* fp = fopen(path, "a");
    if (fp) {
      // every variant's time (a record the loader skips), then the choice
      for (const auto& tv : timed)
        fprintf(fp, "{\"timed\": 1, \"rsize\": %d, \"nb\": %d, \"variant\": %d, \"ms\": %.4f}\n",
                (int)sizeof(R), nb, tv.first, tv.second);
      fprintf(fp, "{\"rsize\": %d, \"nb\": %d, \"variant\": %d, \"ms\": %.4f, \"n\": %lld, \"m\": %d}\n",
              (int)sizeof(R), nb, best, best_ms, (long long)bd.n, m);
      fclose(fp);
    }
  }
  return 0;
}

}  // namespace fb

using namespace fb;

extern "C" int fb_autotune(const fb_band* B, int32_t precision, int32_t nsys, int32_t m,
                           const char* cache_path, int32_t* chosen, double* ms, void* work,
                           size_t* lwork, void* stream) {
  if (check_band(B)) return -1;
  if (precision != 0 && precision != 1) return -2;
  if (nsys < 1) return -3;
  if (m < 1) return -4;
  if (!lwork) return -9;
  hipStream_t st = (hipStream_t)stream;
  if (precision == 1) return autotune_impl<float>(B, nsys, m, cache_path, chosen, ms, work, lwork, st);
  return autotune_impl<double>(B, nsys, m, cache_path, chosen, ms, work, lwork, st);
}

extern "C" int fb_tune_load(const char* cache_path) {
  if (!cache_path) return -1;
  FILE* fp = fopen(cache_path, "r");
  if (!fp) return -1;
  char line[512];
  int n = 0;
  while (fgets(line, sizeof line, fp)) {
    int rs = 0, nb = 0, v = -1;
    if (sscanf(line, " {\"rsize\": %d, \"nb\": %d, \"variant\": %d", &rs, &nb, &v) == 3 &&
        (rs == 4 || rs == 8) && nb > 0 && nb <= 128 && nb % 16 == 0 && v >= 0 &&
        v < kNumVariants) {
      set_tuned_variant((size_t)rs, nb, v);
      ++n;
    }
  }
  fclose(fp);
  return n;
}
