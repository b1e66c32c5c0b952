// Launch timing: HIP events around kernel launches of named classes.
#pragma once
#include "fb_internal.h"

namespace fb {

// Records a start event on construction and a stop event on destruction
// when timing is enabled; work is the algorithmic work of the launch.
// Adds algorithmic work to a class once it is known (launches whose work
// depends on device-side decisions record none themselves).
void prof_add_work(int cls, double work);

struct ProfScope {
  int cls;
  hipStream_t st;
  double work;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int cls, hipStream_t st, double work);
  ~ProfScope();
};

}  // namespace fb
