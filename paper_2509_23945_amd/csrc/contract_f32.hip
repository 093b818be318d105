// Boundary-MPS contraction with environments stored in FP32 (the
// reduced-precision form): the kernels of contract_kernel.h instantiated for
// float storage, in a unit of their own so that the two forms compile in parallel.

#include "contract_kernel.h"

namespace tnmc {

hipError_t launch_contract_f32(const TaskDesc* tasks, int n, int d, int chi_max, hipStream_t s) {
  return launch_contract_et<float>(tasks, n, d, chi_max, s);
}

}  // namespace tnmc
