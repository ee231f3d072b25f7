// Mode-k contraction launches for X stored as double with double arithmetic.
#include "ifctn_device.h"

namespace ifctn {

hipError_t launch_contract_f64(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s) {
  if (a.kind != 0) return fast_dispatch<double, double>(upd, con, spt, a, smem, s);
  return contract_dispatch<double, double>(upd, con, spt, a, smem, s);
}

}  // namespace ifctn
