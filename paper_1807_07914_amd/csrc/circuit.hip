// circuit.hip -- execution of whole gate lists (qsv_apply_circuit) and of
// explicit fused blocks (qsv_apply_fused).
#include "plan.hpp"

namespace qsv {

qsv_status apply_fused_block(qsv_state* s, const qsv_op& o) { return apply_op_pergate(s, o, 0); }

qsv_status run_circuit(qsv_state* s, const qsv_op* ops, int n_ops, const qsv_plan_opts& opts) {
  (void)opts;
  qsv_status st = ensure_workspace(s, dense_ws_bytes());
  if (st) return st;
  for (int i = 0; i < n_ops; ++i) {
    st = apply_op_pergate(s, ops[i], 0);
    if (st) return st;
  }
  return QSV_OK;
}

}  // namespace qsv
