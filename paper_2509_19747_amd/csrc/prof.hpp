// Optional per-kernel timing with HIP events on the launch stream.  Disabled by
// default; when enabled, the launchers of the hot kernels bracket each launch
// with two events (skipped while the stream is being captured into a graph).
#pragma once
#include <hip/hip_runtime.h>

namespace rr {

enum ProfSlot { PROF_KERNEL_MATVEC = 0, PROF_KERNEL_SKETCH, PROF_DENSE_MATVEC, PROF_DENSE_SKETCH,
                PROF_PROJECT, PROF_KERNEL_MATMAT, PROF_KERNEL_MATVEC64, PROF_DENSE_MATVEC64,
                PROF_GROUP_PRODUCT, PROF_GROUP_FINISH, PROF_GROUP_PROJECT, PROF_GROUP_UPDATE, PROF_NSLOTS };

bool prof_enabled();
void prof_record(int slot, hipEvent_t start, hipEvent_t stop);

class ProfScope {
  public:
    ProfScope(int slot, hipStream_t st);
    ~ProfScope();

  private:
    int slot_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace rr
