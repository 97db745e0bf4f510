// RAII bracket of one tracked launch (no-op unless profiling is enabled).
#pragma once
#include <hip/hip_runtime.h>

namespace chaff {
class ProfScope {
  public:
    // work: algorithmic bytes (flops = false) or flops (flops = true) of this launch
    ProfScope(const char* name, hipStream_t st, double work = 0.0, bool flops = false);
    ~ProfScope();

  private:
    hipStream_t st_;
    int rec_ = -1;
};
}  // namespace chaff
