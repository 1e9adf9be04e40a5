// Fusion planning (host): partition an ordered list of operations into blocks that are
// applied as one superoperator each (Sec. 3.3 and its generalisation to k-qubit blocks).
#pragma once

#include <cstdint>
#include <vector>

namespace tanq {

struct PlanOp {
  int j;
  int q[3];
};

struct PlanBlock {
  std::vector<int> qubits;  // block qubits in superoperator local order
  std::vector<int> ops;     // operation indices, circuit order
};

// mode: -1 = no fusion (one block per operation, the op's own qubit order);
//       -2 = the paper's rule: consecutive operations acting on exactly the same ordered
//            qubit tuple are merged (1-qubit runs on one qubit, 2-qubit runs on one ordered
//            pair), nothing else;
//       k in 1..3 = greedy blocks of at most k qubits (sorted ascending).
// Greedy rule: an operation on qubit set Q may join the most recently created block B
// among the last blocks of its qubits when |qubits(B) u Q| <= k.  This is exact: every block
// created after B avoids Q, so the operation commutes past them.  Ties cannot occur (one
// latest block); when it cannot join, it opens a new block.
std::vector<PlanBlock> plan_fusion(const std::vector<PlanOp>& ops, int n, int mode);

}  // namespace tanq
