// Mode-k contraction launches for X stored as bf16x with float arithmetic.
#include "ifctn_device.h"

namespace ifctn {

hipError_t launch_contract_bf16(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s) {
  if (a.kind != 0) return fast_dispatch<bf16x, float>(upd, con, spt, a, smem, s);
  return contract_dispatch<bf16x, float>(upd, con, spt, a, smem, s);
}

}  // namespace ifctn
