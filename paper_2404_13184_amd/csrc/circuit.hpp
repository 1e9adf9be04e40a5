// Host-side circuit records and the device work of fusion, shared by the single-state API
// (api.cpp) and the server (serve.cpp).
#pragma once

#include <cstddef>
#include <memory>
#include <vector>

#include "fuse_plan.hpp"
#include "internal.hpp"

namespace tanq {

// One operation: m Kraus matrices (2^j x 2^j complex, row-major, interleaved) at offset koff
// (doubles) of a matrix pool that may be shared by many operations and circuits.
struct HostOp {
  int j = 0;
  int m = 0;
  int q[3] = {0, 0, 0};
  std::shared_ptr<const std::vector<double>> pool;
  size_t koff = 0;
  const double* K() const { return pool->data() + koff; }
  size_t kdoubles() const { return (size_t)m * ((size_t)1 << (2 * j)) * 2; }
};

struct FusedBlockHost {
  int k = 0;
  int qubits[3] = {0, 0, 0};
  size_t raw_off = 0;   // complex elements
  size_t pack_off = 0;  // bytes
};

inline size_t elem_size(tanq_prec p) { return p == TANQ_F64 ? 16 : 8; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline size_t packed_bytes(int k, tanq_prec p) {
  if (k == 1) return 32 * sizeof(double);
  return (size_t)packed_elems(k) * (p == TANQ_F64 ? sizeof(double) : sizeof(float));
}

std::vector<PlanOp> plan_ops(const std::vector<HostOp>& ops);

// Give every block exactly w qubits by adding qubits it does not act on (the identity there),
// lowest indices first, then sorting.  Needs w <= n.
void widen_plan(std::vector<PlanBlock>& plan, int n, int w);

// Host tables of one fusion: operation and block tables for the kernels, the Kraus pool, the
// per-block host records, and the sizes of the device buffers the kernels need.
struct FuseLayout {
  std::vector<FuseOpDev> ops;
  std::vector<FuseBlockDev> blocks;
  std::vector<double> kraus;  // interleaved complex
  std::vector<FusedBlockHost> host;
  size_t sop_elems = 0;   // complex elements of all operations' superoperators
  size_t raw_elems = 0;   // complex elements of all blocks' FP64 superoperators
  size_t pack_bytes = 0;  // packed operands
  int max_k = 1;
  int count_k[4] = {0, 0, 0, 0};
};

FuseLayout make_fuse_layout(const std::vector<HostOp>& ops, const std::vector<PlanBlock>& plan, tanq_prec p);

// Superoperator construction, FP64 composition and packing on stream s; the tables
// (d_ops, d_blk, d_kraus) must already hold the layout's contents.
void run_fuse_kernels(const FuseLayout& L, const FuseOpDev* d_ops, const FuseBlockDev* d_blk, const double* d_kraus,
                      double* d_sops, double* d_raw, unsigned char* d_packed, tanq_prec p, hipStream_t s);

}  // namespace tanq

struct tanq_circuit_s {
  int n = 0;
  std::vector<tanq::HostOp> ops;
};
