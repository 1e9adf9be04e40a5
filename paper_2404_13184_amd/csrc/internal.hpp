// Internal declarations shared by the host sources and the HIP kernels of libtanq.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tanq.h"

namespace tanq {

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------

struct Error : std::runtime_error {
  tanq_status code;
  Error(tanq_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(tanq_status c, const std::string& m) { throw Error(c, m); }

#define TANQ_HIP(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::tanq::fail(TANQ_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

// ------------------------------------------------------------------------------------
// geometry of one superoperator apply (computed on the host, passed by value)
// ------------------------------------------------------------------------------------

// Tiles: a workgroup owns the 2^V elements of vec(rho) whose "varying" bits take every
// value (the 2k target bits plus the lowest free bits), with the remaining ("fixed") bits
// given by the tile id.  Groups of the superoperator lie wholly inside a tile.
struct ApplyGeom {
  uint64_t ntiles;        // number of tiles = 2^(2n - V)
  uint32_t tj[64];        // tile-local index of each superoperator local index l < 4^k
  uint32_t free_mask;     // tile-local bits that index groups inside the tile
  uint32_t xsrc;          // LDS swizzle: group bits above the bank window ...
  uint32_t xdst;          // ... copied (XOR) into these target-bit positions inside it
  int32_t V;              // tile bits
  int32_t G;              // groups per tile = 2^(V - 2k)
  int32_t nruns;          // runs of fixed bits
  uint8_t vpos[16];       // tile-local bit b -> global bit vpos[b] (ascending)
  uint8_t run_src[8];     // first tile-id bit of run r
  uint8_t run_len[8];     // length of run r
  uint8_t run_dst[8];     // first global bit of run r
};

// One-qubit apply (the paper's C1): groups of 4 at s_i + {0, 2^q, 2^(q+n), 2^q + 2^(q+n)}.
struct C1Geom {
  uint64_t ngroups;  // 4^(n-1)
  int32_t q;
  int32_t n;
};

// A pass: up to kPassMax consecutive 2-qubit superoperators applied to each tile while it is in
// LDS.  The tile holds every target bit of the pass (plus the lowest other bits up to V); the
// LDS swizzle is the linear map S(e) = e ^ (XOR of xcol[b] over the set bits b of e above the
// 256-byte bank window).
constexpr int kPassMax = 8;
// Pass tiles: 2^12 FP64 or 2^13 FP32 elements (64 KiB); superoperators one pass holds (their
// 3M operands must fit in LDS beside two tile buffers).
constexpr int kPassTileBitsF64 = 12, kPassTileBitsF32 = 13;
constexpr int kPassMaxF64 = 4, kPassMaxF32 = 6;
struct PassGeom {
  uint64_t ntiles;               // 2^(2n - V)
  int32_t V;                     // tile bits
  int32_t nruns;                 // runs of fixed bits
  int32_t m;                     // superoperators in the pass
  int32_t pad;
  uint32_t op_off[kPassMax];     // element offset of superoperator j's packed operand
  uint32_t free_mask[kPassMax];  // tile bits that index superoperator j's groups
  uint32_t stj[kPassMax][16];    // S(tile-local index of local index l) of superoperator j
  uint8_t xcol[16];              // swizzle column of each tile bit (0 inside the window)
  uint8_t vpos[16];              // tile bit b -> global bit vpos[b] (ascending)
  uint8_t run_src[16];           // runs of fixed bits (up to 13 around 12 target bits)
  uint8_t run_len[16];
  uint8_t run_dst[16];
};

// Fusion: a block of consecutive operations on at most k qubits.
struct FuseOpDev {
  int32_t j;          // qubits of the operation
  int32_t m;          // Kraus matrices
  int64_t kraus_off;  // offset (complex elements) of K_0 in the Kraus pool
  int64_t sop_off;    // offset (complex elements) of its superoperator in the pool
  int32_t pos[3];     // block-local position of each of its qubits
  int32_t pad;
};

struct FuseBlockDev {
  int32_t k;          // qubits of the block
  int32_t op_begin;   // first operation (index into the op table)
  int32_t op_count;
  int32_t pad;
  int64_t out_off;    // offset (complex elements) of the 4^k x 4^k FP64 result
  int64_t pack_off;   // offset (elements of the packed precision) of the packed operand
};

// Serving: one batched launch applies one superoperator to each of many states.  Items and
// chunks live in device memory; a chunk is a range of tiles of one item.
struct BatchItem {
  uint64_t rho;   // device address of the state
  uint64_t frag;  // device address of the packed operand
  ApplyGeom g;
};

struct BatchChunk {
  uint32_t item;
  uint32_t tile_begin;
  uint32_t tile_end;
  uint32_t pad;
};

// Packed operand sizes (elements of T) per superoperator width.
//   k = 1: 4x4 complex FP64 (32 doubles); k = 2: real-block 32 x 32; k = 3: 3M planar
//   (Sr, Si, Sr + Si) as 4 m-tiles x 16 k-steps x 3 x 64 lanes.
constexpr int packed_elems(int k) { return k == 1 ? 32 : (k == 2 ? 32 * 32 : 4 * 16 * 3 * 64); }

// ------------------------------------------------------------------------------------
// launchers (kernels.hip)
// ------------------------------------------------------------------------------------

ApplyGeom make_apply_geom(int n, int k, const int* qubits, int vbits, tanq_prec p);

// Apply-kernel variants per (k, precision), k in {2, 3}: count, shape, process-wide choice.
int variant_count(int k, tanq_prec p);
bool variant_describe(int k, tanq_prec p, int index, int* tile_bits, int* threads, int* staging);
bool variant_select(int k, tanq_prec p, int index);
int variant_selected(int k, tanq_prec p);
// autotuned variant per (n, k, precision); -1 = none (the process-wide choice applies)
constexpr int kTunedMaxN = 17;
bool variant_tune(int n, int k, tanq_prec p, int index);
int variant_tuned(int n, int k, tanq_prec p);
int variant_for(int n, int k, tanq_prec p);
int variant_find(int k, tanq_prec p, int tile_bits, int threads, int staging);
void launch_apply_variant(void* rho, int n, tanq_prec p, int k, int index, const int* qubits, const void* packed,
                          hipStream_t s);

// Passes (pass.hip): tile bits per precision; geometry of m superoperators (qubits: m pairs,
// op_off: element offsets of their packed operands); launch on one state.
int pass_tile_bits(tanq_prec p);
// Most superoperators one pass of precision p holds (at most kPassMax).
int pass_max(tanq_prec p);
// conflict_free (optional): access patterns (two per superoperator) whose LDS reads and writes
// are free of bank conflicts under the chosen swizzle; achievable (optional): an upper bound of
// that count over all swizzles of this form.
PassGeom make_pass_geom(int n, int m, const int* qubits, const uint32_t* op_off, tanq_prec p,
                        int* conflict_free = nullptr, int* achievable = nullptr);
void launch_pass(void* rho, tanq_prec p, const PassGeom& g, const void* frags, hipStream_t s);
// Process-wide limit on superoperators per pass (1 = no passes).
int pass_limit();
void set_pass_limit(int m);

void launch_init_zero(void* rho, int n, tanq_prec p, hipStream_t s);
void launch_gather(const void* rho, tanq_prec p, const uint64_t* idx_dev, size_t count, void* out_dev,
                   hipStream_t s);
void launch_fill_random(void* rho, int n, tanq_prec p, uint64_t seed, hipStream_t s);
void launch_scale(void* rho, int n, tanq_prec p, double f, hipStream_t s);
// Sustained matrix-unit rate (TFLOP/s) of the pass kernels' multiplication loop shape on the
// current device; synchronous.
double mfma_rate_tflops(tanq_prec p);

// All-qubit sampling (tanq_sample and its variant without allocations): argument checks (also
// returning the handle's qubit count and device), and the work itself on the caller's device
// buffers for the CDF (2^n doubles) and the outcomes (shots words); synchronises.
void sample_check(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10, uint64_t* host_out,
                  int* n, int* device);
void sample_run(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10, double* cdf_dev,
                uint64_t* out_dev, uint64_t* host_out);

// Apply one superoperator whose packed operand is at `packed` (device).
//   k == 1: packed = 4x4 complex FP64 (32 doubles), used for both precisions.
//   k == 2, 3: packed = real-block fragments in precision p.
void launch_apply(void* rho, int n, tanq_prec p, int k, const int* qubits, const void* packed,
                  hipStream_t s);

// Superoperators of every operation (sum_i conj(K_i) (x) K_i), FP64.
void launch_build_superops(const FuseOpDev* ops, int nops, const double* kraus, double* sops,
                           hipStream_t s);
// Compose each block's superoperators in circuit order (FP64) into `out`.
void launch_compose(const FuseBlockDev* blocks, int nblocks, int max_k, const FuseOpDev* ops,
                    const double* sops, double* out, hipStream_t s);
// Pack FP64 block superoperators into the apply kernels' operand layout.
void launch_pack(const FuseBlockDev* blocks, int nblocks, const double* raw, void* packed,
                 tanq_prec p, hipStream_t s);
// Pack a single FP64 superoperator (device) of width k.
void launch_pack_one(int k, const double* raw, void* packed, tanq_prec p, hipStream_t s);

// Reductions (FP64).  partials: device scratch of at least reduce_partials() doubles.
int reduce_partials();
void launch_diag(const void* rho, int n, tanq_prec p, double* probs_dev, double* partials,
                 double* result_dev, int renormalize, hipStream_t s);
void launch_pauli(const void* rho, int n, tanq_prec p, int count, const uint64_t* masks_dev,
                  double* partials, double* result_dev, hipStream_t s);

// vec(rho) = e_idx (rho = |r><c| for idx = r + c 2^n)
void launch_init_basis(void* rho, int n, tanq_prec p, uint64_t idx, hipStream_t s);
// Reduced density matrix on k <= 4 kept qubits (device list keep_dev); out_dev: 2 * 4^k doubles
void launch_reduced(const void* rho, int n, tanq_prec p, int k, const int* keep_dev, double* out_dev, hipStream_t s);

// Classical readout error on the probability vector, one qubit at a time (host arrays p01,
// p10 of n values), in place.
void launch_readout(double* probs_dev, int n, const double* p01, const double* p10, hipStream_t s);
// Inverse-CDF sampling of `shots` outcomes with SplitMix64 draws; cdf_dev: 2^n doubles.
void launch_sample(const double* probs_dev, int n, double* cdf_dev, uint64_t shots, uint64_t seed, uint64_t* out_dev,
                   hipStream_t s);

// out3 = (||a-b||_F, max|a-b|, ||a||_F); partials: reduce_partials() doubles.
void launch_compare(const void* a, tanq_prec pa, const void* b, tanq_prec pb, uint64_t nel, double* partials,
                    double* result_dev, hipStream_t s);

int device_cu_count();

// Tile bits of the batched kernel for width k (2 or 3) and precision p (geometry of the items
// must be built with this value).
int batch_tile_bits(int k, tanq_prec p);
// Workgroups of the batched kernel's persistent grid on the current device.
int batch_grid(int k, tanq_prec p);
// Apply the items of `*count` chunks (count lives in device memory so the launch can be
// captured in a graph and replayed with new contents).
void launch_batch(int k, tanq_prec p, const BatchItem* items, const BatchChunk* chunks, uint32_t* count,
                  hipStream_t s);

}  // namespace tanq
