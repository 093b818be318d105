// Boundary-MPS contraction: the kernels of contract_kernel.h instantiated
// with environments stored in FP32 (the reduced-precision form) and the
// products on the vector ALU, in a unit of their own so that the instantiations compile in parallel.

#include "contract_kernel.h"

namespace tnmc {

hipError_t launch_contract_f32(const TaskDesc* tasks, int n, int d, int chi_max, int full, hipStream_t s) {
  return launch_contract_et<float, false>(tasks, n, d, chi_max, full, s);
}

}  // namespace tnmc
