// Instantiations of the single-problem MTTKRP kernels for float tensors with
// 4-entry lane loads (kept in a translation unit of their own so the kernel
// variants compile in parallel).
#include "mttkrp_kernels.hpp"

namespace cpamg {

namespace {

template <typename T, int NT, int VW, bool BL>
static const void* kernel_ptr(int kind, int tw, bool vec, bool ys) {
  if (kind == 1)
    return vec ? (const void*)mttkrp_kind1<T, NT, VW, true, BL> : (const void*)mttkrp_kind1<T, NT, VW, false, BL>;
  const bool k3 = kind == 3;
  if (!k3 && ys) {   // mode 1 storing the stage-1 tiles (dimension tree)
    if (tw == 4 && NT == 1)
      return vec ? (const void*)mttkrp_kind23<T, 1, 4, false, VW, true, BL, true>
                 : (const void*)mttkrp_kind23<T, 1, 4, false, VW, false, BL, true>;
    return vec ? (const void*)mttkrp_kind23<T, NT, 2, false, VW, true, BL, true>
               : (const void*)mttkrp_kind23<T, NT, 2, false, VW, false, BL, true>;
  }
  if (tw == 4 && NT == 1) {
    if (k3) return vec ? (const void*)mttkrp_kind23<T, 1, 4, true, VW, true, BL> : (const void*)mttkrp_kind23<T, 1, 4, true, VW, false, BL>;
    return vec ? (const void*)mttkrp_kind23<T, 1, 4, false, VW, true, BL> : (const void*)mttkrp_kind23<T, 1, 4, false, VW, false, BL>;
  }
  if (k3) return vec ? (const void*)mttkrp_kind23<T, NT, 2, true, VW, true, BL> : (const void*)mttkrp_kind23<T, NT, 2, true, VW, false, BL>;
  return vec ? (const void*)mttkrp_kind23<T, NT, 2, false, VW, true, BL> : (const void*)mttkrp_kind23<T, NT, 2, false, VW, false, BL>;
}

}  // namespace

const void* mttkrp_kernel_f32v4(const MttkrpPlan& p, bool vec, bool ys) {
  if (p.bl) return p.nt == 1 ? kernel_ptr<float, 1, 4, true>(p.kind, p.tw, vec, ys) : kernel_ptr<float, 2, 4, true>(p.kind, p.tw, vec, ys);
  return p.nt == 1 ? kernel_ptr<float, 1, 4, false>(p.kind, p.tw, vec, ys) : kernel_ptr<float, 2, 4, false>(p.kind, p.tw, vec, ys);
}

}  // namespace cpamg
