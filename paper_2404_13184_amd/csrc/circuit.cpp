#include "circuit.hpp"

#include <algorithm>
#include <map>
#include <utility>

namespace tanq {

std::vector<PlanOp> plan_ops(const std::vector<HostOp>& ops) {
  std::vector<PlanOp> p(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    p[i].j = ops[i].j;
    for (int t = 0; t < 3; ++t) p[i].q[t] = ops[i].q[t];
  }
  return p;
}

void widen_plan(std::vector<PlanBlock>& plan, int n, int w) {
  for (auto& b : plan) {
    for (int q = 0; q < n && (int)b.qubits.size() < w; ++q)
      if (std::find(b.qubits.begin(), b.qubits.end(), q) == b.qubits.end()) b.qubits.push_back(q);
    std::sort(b.qubits.begin(), b.qubits.end());
  }
}

FuseLayout make_fuse_layout(const std::vector<HostOp>& ops, const std::vector<PlanBlock>& plan, tanq_prec p) {
  FuseLayout L;
  // identical Kraus sets (same pool and offset, e.g. a noise channel repeated through a
  // circuit) are uploaded once; their superoperators are still built per operation
  std::map<std::pair<const void*, size_t>, int64_t> seen;
  for (const auto& pb : plan) {
    const int k = (int)pb.qubits.size();
    if (k > 3) fail(TANQ_E_UNSUPPORTED, "a block wider than 3 qubits");
    L.max_k = std::max(L.max_k, k);
    FuseBlockDev bd{};
    bd.k = k;
    bd.op_begin = (int)L.ops.size();
    bd.op_count = (int)pb.ops.size();
    bd.out_off = (int64_t)L.raw_elems;
    bd.pack_off = (int64_t)L.pack_bytes;
    FusedBlockHost bh;
    bh.k = k;
    for (int t = 0; t < k; ++t) bh.qubits[t] = pb.qubits[t];
    bh.raw_off = L.raw_elems;
    bh.pack_off = L.pack_bytes;
    L.raw_elems += (size_t)1 << (4 * k);
    L.pack_bytes += align256(packed_bytes(k, p));
    for (int oi : pb.ops) {
      const HostOp& ho = ops[oi];
      FuseOpDev od{};
      od.j = ho.j;
      od.m = ho.m;
      const auto key = std::make_pair((const void*)ho.pool.get(), ho.koff);
      auto it = seen.find(key);
      if (it == seen.end()) {
        it = seen.emplace(key, (int64_t)(L.kraus.size() / 2)).first;
        L.kraus.insert(L.kraus.end(), ho.K(), ho.K() + ho.kdoubles());
      }
      od.kraus_off = it->second;
      od.sop_off = (int64_t)L.sop_elems;
      for (int t = 0; t < ho.j; ++t) {
        int pos = -1;
        for (int u = 0; u < k; ++u)
          if (pb.qubits[u] == ho.q[t]) pos = u;
        if (pos < 0) fail(TANQ_E_STATE, "operation qubit outside its block");
        od.pos[t] = pos;
      }
      L.sop_elems += (size_t)1 << (4 * ho.j);
      L.ops.push_back(od);
    }
    L.blocks.push_back(bd);
    L.host.push_back(bh);
    L.count_k[k] += 1;
  }
  return L;
}

void run_fuse_kernels(const FuseLayout& L, const FuseOpDev* d_ops, const FuseBlockDev* d_blk, const double* d_kraus,
                      double* d_sops, double* d_raw, unsigned char* d_packed, tanq_prec p, hipStream_t s) {
  if (L.blocks.empty()) return;
  launch_build_superops(d_ops, (int)L.ops.size(), d_kraus, d_sops, s);
  launch_compose(d_blk, (int)L.blocks.size(), L.max_k, d_ops, d_sops, d_raw, s);
  launch_pack(d_blk, (int)L.blocks.size(), d_raw, d_packed, p, s);
}

}  // namespace tanq
