// kernels_f32.hip -- the kernel variants of the float field table (sweep,
// refresh, batch/serve); see kernels.hpp.
#include <hip/hip_runtime.h>

#define PTMI_KERNEL_SELECT
#include "kernels.hpp"

namespace ptmi {

const void *sweep_kernel_f32(int q, const LdsPlan &p) { return sweep_fn<float>(q, p); }
const void *refresh_kernel_f32(const LdsPlan &p) { return refresh_fn<float>(p); }
const void *jobs_kernel_f32() { return reinterpret_cast<const void *>(&k_jobs<float>); }

}  // namespace ptmi
