// RAII bracket of one tracked launch (no-op unless profiling is enabled).
#pragma once
#include <hip/hip_runtime.h>

namespace chaff {
// Algorithmic work of one launch: HBM bytes the method must move and the flops
// it must do (0 where a figure is not stated).
struct ProfWork {
    double bytes, flops;
};
class ProfScope {
  public:
    // work: algorithmic bytes (flops = false) or flops (flops = true) of this launch
    ProfScope(const char* name, hipStream_t st, double work = 0.0, bool flops = false)
        : ProfScope(name, st, flops ? ProfWork{0.0, work} : ProfWork{work, 0.0}) {}
    ProfScope(const char* name, hipStream_t st, ProfWork w);
    ~ProfScope();

  private:
    hipStream_t st_;
    int rec_ = -1;
};
}  // namespace chaff
