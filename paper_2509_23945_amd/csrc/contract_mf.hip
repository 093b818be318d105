// Boundary-MPS contraction: the kernels of contract_kernel.h instantiated
// with FP64 environments and the products on the matrix cores (FP64 MFMA), in a unit of their own so that the instantiations compile in parallel.

#include "contract_kernel.h"

namespace tnmc {

hipError_t launch_contract_f64_mf(const TaskDesc* tasks, int n, int d, int chi_max, int full, hipStream_t s) {
  return launch_contract_et<double, true>(tasks, n, d, chi_max, full, s);
}

}  // namespace tnmc
