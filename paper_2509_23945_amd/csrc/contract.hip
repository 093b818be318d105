// Boundary-MPS contraction (SM S1.B): the kernels are in contract_kernel.h;
// this unit instantiates them for FP64 environments and holds the dispatch.

#include "contract_kernel.h"

namespace tnmc {

int g_force_retry = 0;
int g_layout_full[2][2] = {{0, 0}, {0, 0}};

void set_force_retry(int on) { g_force_retry = on; }

// Whether a (d, chi_max) class runs the compact layout (two tasks per CU)
// by default: the same test as launch_contract_t's.
template <int DP, int CHIM>
constexpr bool has_compact() {
  return sizeof(double) * Layout<DP, CHIM, false>::total > kHalfLds &&
         sizeof(double) * Layout<DP, CHIM, true>::total <= kHalfLds;
}
bool contract_has_compact(int d, int chi_max) {
  if (d == 2) {
    switch (chi_max) {
      case 4: return has_compact<2, 4>();
      case 8: return has_compact<2, 8>();
      case 16: return has_compact<2, 16>();
      case 32: return has_compact<2, 32>();
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return has_compact<3, 4>();
      case 8: return has_compact<3, 8>();
      case 16: return has_compact<3, 16>();
      case 32: return has_compact<3, 32>();
    }
  }
  return false;
}
void set_layout_full(int d, int precision, int full) { g_layout_full[d == 3][precision == kPrecF32] = full ? 1 : 0; }

// Bytes of the full tile layout: the LDS of a full-layout workgroup, and the
// per-task global scratch of the retry path (and of d = 3, chi = 32, whose
// tiles always live there); independent of the environment storage type.
size_t contract_lds_bytes(int d, int chi_max) {
  if (d == 2) {
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<2, 4>::total;
      case 8: return sizeof(double) * Layout<2, 8>::total;
      case 16: return sizeof(double) * Layout<2, 16>::total;
      case 32: return sizeof(double) * Layout<2, 32>::total;
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<3, 4>::total;
      case 8: return sizeof(double) * Layout<3, 8>::total;
      case 16: return sizeof(double) * Layout<3, 16>::total;
      case 32: return sizeof(double) * Layout<3, 32>::total;
    }
  }
  return 0;
}

bool contract_supported(int d, int chi_max) { return contract_lds_bytes(d, chi_max) != 0; }

// Whether the (d, chi_max) contraction keeps its tiles in per-task global
// scratch (its full layout exceeds a CU's LDS).
bool contract_uses_global(int d, int chi_max) { return contract_lds_bytes(d, chi_max) > kCuLds; }

int chi_bucket(int chi) {
  if (chi <= 4) return 4;
  if (chi <= 8) return 8;
  if (chi <= 16) return 16;
  if (chi <= 32) return 32;
  return 0;
}

hipError_t launch_contract(const TaskDesc* tasks, int n, int d, int chi_max, int precision, hipStream_t s) {
  if (precision == kPrecF32) return launch_contract_f32(tasks, n, d, chi_max, s);
  return launch_contract_et<double>(tasks, n, d, chi_max, s);
}

}  // namespace tnmc
