// Four-Russians XOR-PIR kernel (placeholder until implemented).
#include <hip/hip_runtime.h>

#include "engine.h"

namespace talek {

bool m4r_plan_supported(const Plan &) { return false; }

uint32_t m4r_tasks(const ReadGeom &, const Plan &) { return 1; }

hipError_t launch_m4r_read(const ReadGeom &, const Plan &, void *, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace talek
