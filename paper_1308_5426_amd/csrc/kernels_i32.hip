// kernels_i32.hip -- the kernel variants of the int32_t field table (sweep,
// refresh, batch/serve); see kernels.hpp.
#include <hip/hip_runtime.h>

#define PTMI_KERNEL_SELECT
#include "kernels.hpp"

namespace ptmi {

const void *sweep_kernel_i32(int q, const LdsPlan &p) { return sweep_fn<int32_t>(q, p); }
const void *refresh_kernel_i32(const LdsPlan &p) { return refresh_fn<int32_t>(p); }
const void *jobs_kernel_i32() { return reinterpret_cast<const void *>(&k_jobs<int32_t>); }

}  // namespace ptmi
