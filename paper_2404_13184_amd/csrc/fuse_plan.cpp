#include "fuse_plan.hpp"

#include <algorithm>

namespace tanq {

std::vector<PlanBlock> plan_fusion(const std::vector<PlanOp>& ops, int n, int mode) {
  std::vector<PlanBlock> blocks;
  std::vector<int> last(n, -1);  // latest block touching each qubit
  for (int i = 0; i < (int)ops.size(); ++i) {
    const PlanOp& op = ops[i];
    int target = -1;
    for (int t = 0; t < op.j; ++t) target = std::max(target, last[op.q[t]]);

    bool joined = false;
    if (target >= 0 && mode != -1) {
      PlanBlock& B = blocks[target];
      if (mode == -2) {
        // same ordered tuple, and B must be the last block of every qubit of the op
        bool same = (int)B.qubits.size() == op.j;
        for (int t = 0; same && t < op.j; ++t) same = B.qubits[t] == op.q[t] && last[op.q[t]] == target;
        if (same) {
          B.ops.push_back(i);
          joined = true;
        }
      } else {
        std::vector<int> u = B.qubits;
        for (int t = 0; t < op.j; ++t)
          if (std::find(u.begin(), u.end(), op.q[t]) == u.end()) u.push_back(op.q[t]);
        if ((int)u.size() <= mode) {
          std::sort(u.begin(), u.end());
          B.qubits = u;
          B.ops.push_back(i);
          joined = true;
        }
      }
    }
    if (!joined) {
      PlanBlock nb;
      nb.qubits.assign(op.q, op.q + op.j);
      if (mode > 0) std::sort(nb.qubits.begin(), nb.qubits.end());
      nb.ops.push_back(i);
      blocks.push_back(std::move(nb));
      target = (int)blocks.size() - 1;
    }
    for (int t = 0; t < op.j; ++t) last[op.q[t]] = target;
  }
  return blocks;
}

}  // namespace tanq
