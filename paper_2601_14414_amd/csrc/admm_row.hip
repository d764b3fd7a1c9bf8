// admm_row.hip -- row-per-lane ADMM kernel for long single horizons.
#include <hip/hip_runtime.h>

#include "pimpc_row.hpp"

namespace pimpc {

bool row_supported(int, int, int, int, int) { return false; }
size_t row_scratch_bytes(const InstDev&, int) { return 0; }
hipError_t row_prepare(int, const InstDev&) { return hipSuccess; }
hipError_t launch_row(int, const RowArgs*, const InstDev&, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace pimpc
