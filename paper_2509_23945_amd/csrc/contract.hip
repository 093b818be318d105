// Boundary-MPS contraction (SM S1.B): the kernels are in contract_kernel.h;
// this unit instantiates them for FP64 environments with the products on the
// vector ALU, and holds the dispatch over storage precision and product engine
// (the other instantiations are in units of their own, which compile in
// parallel).

#include "contract_kernel.h"

namespace tnmc {

int g_force_retry = 0;

int g_force_narrow = 0;

void set_force_retry(int on) { g_force_retry = on; }
void set_force_narrow(int on) { g_force_narrow = on; }

int device_cus() {
  static int cus = 0;
  if (cus <= 0) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cus = c;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

bool contract_has_compact(int d, int chi_max) {
  if (d == 2) {
    switch (chi_max) {
      case 4: return layout_has_compact<2, 4>();
      case 8: return layout_has_compact<2, 8>();
      case 16: return layout_has_compact<2, 16>();
      case 32: return layout_has_compact<2, 32>();
      case 64: return layout_has_compact<2, 64>();
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return layout_has_compact<3, 4>();
      case 8: return layout_has_compact<3, 8>();
      case 16: return layout_has_compact<3, 16>();
      case 32: return layout_has_compact<3, 32>();
    }
  } else if (d == 4) {
    switch (chi_max) {
      case 4: return layout_has_compact<4, 4>();
      case 8: return layout_has_compact<4, 8>();
    }
  }
  return false;
}

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
      case 64: return sizeof(double) * Layout<2, 64>::total;
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<3, 4>::total;
      case 8: return sizeof(double) * Layout<3, 8>::total;
      case 16: return sizeof(double) * Layout<3, 16>::total;
      case 32: return sizeof(double) * Layout<3, 32>::total;
    }
  } else if (d == 4) {   // TNMCMC-2 composite layers (superspins), chi <= 8
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<4, 4>::total;
      case 8: return sizeof(double) * Layout<4, 8>::total;
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
  if (chi <= 64) return 64;
  return 0;
}

hipError_t launch_contract_f64(const TaskDesc* tasks, int n, int d, int chi_max, int full, hipStream_t s) {
  return launch_contract_et<double, false>(tasks, n, d, chi_max, full, s);
}

hipError_t launch_contract(const TaskDesc* tasks, int n, int d, int chi_max, int precision, ContractCfg cfg,
                           hipStream_t s) {
  // chi_max = 64 (tiles in global memory) and the superspin layers are built
  // with vector-ALU products only
  if (chi_max == 64 || d == 4) cfg.mfma = 0;
  if (precision == kPrecF32)
    return cfg.mfma ? launch_contract_f32_mf(tasks, n, d, chi_max, cfg.full, s)
                    : launch_contract_f32(tasks, n, d, chi_max, cfg.full, s);
  return cfg.mfma ? launch_contract_f64_mf(tasks, n, d, chi_max, cfg.full, s)
                  : launch_contract_f64(tasks, n, d, chi_max, cfg.full, s);
}

}  // namespace tnmc
