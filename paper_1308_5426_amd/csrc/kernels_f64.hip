// kernels_f64.hip -- the kernel variants of the double field table (sweep,
// refresh, batch/serve); see kernels.hpp.
#include <hip/hip_runtime.h>

#define PTMI_KERNEL_SELECT
#include "kernels.hpp"

namespace ptmi {

const void *sweep_kernel_f64(int q, const LdsPlan &p) { return sweep_fn<double>(q, p); }
const void *refresh_kernel_f64(const LdsPlan &p) { return refresh_fn<double>(p); }
const void *jobs_kernel_f64() { return reinterpret_cast<const void *>(&k_jobs<double>); }

}  // namespace ptmi
