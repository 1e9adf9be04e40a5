// Batched superoperator apply for the serving loop (gfx950): one launch applies the next fused
// superoperator of every active request to that request's own vec(rho).  The work is a list of
// chunks (request item, range of tiles); a persistent grid claims chunks from the list one at
// a time (an atomic counter in the work list), stages each item's tile geometry in LDS (its run
// table and row offsets in scalar registers) and runs the same tile multiplication as the
// single-state kernels (tile.hpp).  States of different requests are disjoint, so the chunks
// of one launch are independent; successive launches are ordered on the stream.  The number of
// chunks is read from device memory, which lets a fixed launch be captured in a graph and
// replayed.
#include <type_traits>

#include "tile.hpp"

namespace tanq {

// The run table of the current item (the tile id -> global offset map), read once per item
// from its geometry in LDS into scalar registers: the single-state kernels have it in their
// kernel arguments, here it would otherwise be re-read from LDS for every tile.
struct BatchRuns {
  uint32_t src[2], len[2], dst[2];  // run r's byte r % 4 of word r / 4
  int32_t n;

  template <typename G>
  __device__ inline void load(const G& g) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      src[w] = (uint32_t)__builtin_amdgcn_readfirstlane((int)reinterpret_cast<const uint32_t*>(g.run_src)[w]);
      len[w] = (uint32_t)__builtin_amdgcn_readfirstlane((int)reinterpret_cast<const uint32_t*>(g.run_len)[w]);
      dst[w] = (uint32_t)__builtin_amdgcn_readfirstlane((int)reinterpret_cast<const uint32_t*>(g.run_dst)[w]);
    }
    n = __builtin_amdgcn_readfirstlane(g.nruns);
  }

  // the same map as tile_base(g, tile)
  __device__ inline uint64_t base(uint64_t tile) const {
    uint64_t b = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r < n) {
        const uint32_t sh = 8 * (r % 4);
        const uint32_t rs = (src[r / 4] >> sh) & 0xffu, rl = (len[r / 4] >> sh) & 0xffu, rd = (dst[r / 4] >> sh) & 0xffu;
        b |= ((tile >> rs) & ((1ull << rl) - 1ull)) << rd;
      }
    return b;
  }
};

// The tiles [t0, t1) of one item, in place: the next tile is prefetched into registers while
// the current one is multiplied in LDS, as in the single-state kernel.
template <bool FULL, typename T, typename IO, typename Op, typename G>
__device__ inline void batch_tiles(T* __restrict__ rho, const IO& io, const Op& op, const G& g, const BatchRuns& runs,
                                   u32x4* lds, uint32_t t0, uint32_t t1, int tid, int lane, int wave) {
  using c2 = typename Mfma<T>::c2;
  uint64_t cur = runs.base(t0);
  u32x4 buf[IO::ITERS];
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) buf[it] = *global_ptr(reinterpret_cast<const u32x4*>(rho + 2 * (cur + io.off[it])));
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) lds[io.lslot[it]] = buf[it];
  lds_barrier();
  for (uint32_t t = t0;;) {
    const bool more = t + 1 < t1;
    uint64_t nbase = 0;
    if (more) {
      nbase = runs.base(t + 1);
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.template has<FULL>(it, tid))
          buf[it] = *global_ptr(reinterpret_cast<const u32x4*>(rho + 2 * (nbase + io.off[it])));
    }
    if constexpr (std::is_same_v<Op, Op2<T, Op::kVmax, Op::kThreads>>)
      op.template compute<FULL>(reinterpret_cast<T*>(lds), g, lane, wave);
    else
      op.template compute<FULL>(reinterpret_cast<c2*>(lds), g, lane, wave);
    lds_barrier();
#pragma unroll
    for (int it = 0; it < IO::ITERS; ++it)
      if (io.template has<FULL>(it, tid)) *global_ptr(reinterpret_cast<u32x4*>(rho + 2 * (cur + io.off[it]))) = lds[io.lslot[it]];
    lds_barrier();  // every store-phase LDS read is done before the next tile lands (or the next chunk)
    if (!more) break;
#pragma unroll
    for (int it = 0; it < IO::ITERS; ++it)
      if (io.template has<FULL>(it, tid)) lds[io.lslot[it]] = buf[it];
    lds_barrier();
    ++t;
    cur = nbase;
  }
}

// k = 3: the tiles [t0, t1) of one item with two LDS buffers.  Each tile is multiplied out of
// place from `in` into `out` (every wave reads the whole tile, so in place would need a barrier
// between the reads and the writes); one barrier then separates the multiplication from the
// store of `out` and the refill of `in` with the next tile (prefetched into registers), and a
// second one the refill from the next multiplication.
template <bool FULL, typename T, typename IO, typename Op, typename G>
__device__ inline void batch_tiles_oop(T* __restrict__ rho, const IO& io, const Op& op, const G& g,
                                       const BatchRuns& runs, u32x4* in, u32x4* out, uint32_t t0, uint32_t t1, int tid,
                                       int lane, int wave) {
  using c2 = typename Mfma<T>::c2;
  uint64_t cur = runs.base(t0);
  u32x4 buf[IO::ITERS];
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) buf[it] = *global_ptr(reinterpret_cast<const u32x4*>(rho + 2 * (cur + io.off[it])));
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) in[io.lslot[it]] = buf[it];
  lds_barrier();
  for (uint32_t t = t0;;) {
    const bool more = t + 1 < t1;
    uint64_t nbase = 0;
    if (more) {
      nbase = runs.base(t + 1);
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.template has<FULL>(it, tid))
          buf[it] = *global_ptr(reinterpret_cast<const u32x4*>(rho + 2 * (nbase + io.off[it])));
    }
    op.template compute_to<FULL>(reinterpret_cast<const c2*>(in), reinterpret_cast<c2*>(out), g, lane, wave);
    lds_barrier();  // results complete; `in` is no longer read
#pragma unroll
    for (int it = 0; it < IO::ITERS; ++it)
      if (io.template has<FULL>(it, tid)) *global_ptr(reinterpret_cast<u32x4*>(rho + 2 * (cur + io.off[it]))) = out[io.lslot[it]];
    if (more) {
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.template has<FULL>(it, tid)) in[io.lslot[it]] = buf[it];
    }
    lds_barrier();  // `out` read out and `in` refilled (or, after the last tile, free for the next chunk)
    if (!more) break;
    ++t;
    cur = nbase;
  }
}

// Workgroups per CU the FP32 k = 3 kernel is compiled for: three (at most 168 registers per lane,
// a few of them spilled outside the multiplication) instead of the two its unconstrained
// allocation allows; the third workgroup's waves hide the others' barriers and tile turnovers
// (measured on the serving stream's latency and throughput; four, at 128 registers, spills
// inside the loop).  Every other shape keeps its allocation.
template <typename T, int K>
struct BatchMinBlocks { static constexpr int value = 1; };
template <>
struct BatchMinBlocks<float, 3> { static constexpr int value = 3; };

template <typename T, int K, int VMAX, int NT>
__global__ __launch_bounds__(NT, (BatchMinBlocks<T, K>::value)) void batch_apply_kernel(const BatchItem* __restrict__ items,
                                                         const BatchChunk* __restrict__ chunks,
                                                         uint32_t* __restrict__ count) {
  using IO = TileIo<T, VMAX, NT>;
  using Op = std::conditional_t<K == 2, Op2<T, VMAX, NT>, Op3<T, VMAX, NT>>;
  static_assert(sizeof(ApplyGeom) % 4 == 0, "geometry copied as dwords");

  __shared__ u32x4 lds[IO::SLOTS];
  // FP32 k = 3: the out-of-place result buffer (FP64 k = 3 stays in place: its operand slices
  // leave no registers for the second path)
  constexpr bool kOop = K == 3 && std::is_same_v<T, float>;
  __shared__ u32x4 lds2[kOop ? IO::SLOTS : 1];
  __shared__ ApplyGeom sg;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nch = count[0];
  __shared__ uint32_t s_next;

  uint32_t cur = 0xffffffffu;
  bool full = false;
  IO io;
  Op op;
  BatchRuns runs;
  T* rho = nullptr;
  for (;;) {
    // dynamic assignment: each workgroup claims the next chunk (count[1], zeroed by the copy of
    // the work list that precedes every launch), so the launch ends when its last chunks do
    if (tid == 0) s_next = atomicAdd(&count[1], 1u);
    lds_barrier();
    const uint32_t c = s_next;
    lds_barrier();
    if (c >= nch) break;
    const BatchChunk ch = chunks[c];
    if (ch.item != cur) {
      lds_barrier();  // the previous item's geometry is no longer read
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&items[ch.item].g);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sg);
      for (int i = tid; i < (int)(sizeof(ApplyGeom) / 4); i += NT) dst[i] = src[i];
      lds_barrier();
      rho = reinterpret_cast<T*>(items[ch.item].rho);
      const T* frag = reinterpret_cast<const T*>(items[ch.item].frag);
      io.init(sg, tid);
      if constexpr (K == 2)
        op.load(frag, lane);
      else
        op.load(frag, lane, wave);
      op.prepare(sg, lane, wave);
      runs.load(sg);
      full = __builtin_amdgcn_readfirstlane(sg.V) == VMAX;
      cur = ch.item;
    }
    if (ch.tile_begin >= ch.tile_end) continue;
    if constexpr (kOop) {
      if (full)
        batch_tiles_oop<true, T>(rho, io, op, sg, runs, lds, lds2, ch.tile_begin, ch.tile_end, tid, lane, wave);
      else
        batch_tiles_oop<false, T>(rho, io, op, sg, runs, lds, lds2, ch.tile_begin, ch.tile_end, tid, lane, wave);
    } else {
      if (full)
        batch_tiles<true, T>(rho, io, op, sg, runs, lds, ch.tile_begin, ch.tile_end, tid, lane, wave);
      else
        batch_tiles<false, T>(rho, io, op, sg, runs, lds, ch.tile_begin, ch.tile_end, tid, lane, wave);
    }
  }
}

// Shapes: 16 KiB tiles for k = 2 (2^10 FP64 / 2^11 FP32 elements) and for FP32 k = 3 (2^11
// elements, 256 threads: measured 4% more circuits/s on the serving stream than 2^12 / 512);
// FP64 k = 3 uses 2^11 elements and 512 threads, which keeps it free of register spills.
template <typename T, int K>
struct BatchShape;
template <>
struct BatchShape<double, 2> { static constexpr int V = 10, NT = 256; };
template <>
struct BatchShape<float, 2> { static constexpr int V = 11, NT = 256; };
template <>
struct BatchShape<double, 3> { static constexpr int V = 11, NT = 512; };
template <>
struct BatchShape<float, 3> { static constexpr int V = 11, NT = 256; };

int batch_tile_bits(int k, tanq_prec p) {
  if (k == 2) return p == TANQ_F64 ? BatchShape<double, 2>::V : BatchShape<float, 2>::V;
  return p == TANQ_F64 ? BatchShape<double, 3>::V : BatchShape<float, 3>::V;
}

// Persistent grid of the batched kernel: as many workgroups as fit on the device at once.
template <typename T, int K>
static unsigned batch_grid_typed() {
  constexpr int NT = BatchShape<T, K>::NT;
  static thread_local int cap_dev = -1;
  static thread_local unsigned cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (cap_dev != dev) {
    int per_cu = 0;
    TANQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, batch_apply_kernel<T, K, BatchShape<T, K>::V, NT>, NT, 0));
    cap = (unsigned)(device_cu_count() * (per_cu < 1 ? 1 : per_cu));
    cap_dev = dev;
  }
  return cap;
}

int batch_grid(int k, tanq_prec p) {
  if (k == 2) return (int)(p == TANQ_F64 ? batch_grid_typed<double, 2>() : batch_grid_typed<float, 2>());
  if (k == 3) return (int)(p == TANQ_F64 ? batch_grid_typed<double, 3>() : batch_grid_typed<float, 3>());
  fail(TANQ_E_ARG, "batched width must be 2 or 3");
}

template <typename T, int K>
static void launch_batch_typed(const BatchItem* items, const BatchChunk* chunks, uint32_t* count,
                               hipStream_t s) {
  constexpr int V = BatchShape<T, K>::V, NT = BatchShape<T, K>::NT;
  hipLaunchKernelGGL((batch_apply_kernel<T, K, V, NT>), dim3(batch_grid_typed<T, K>()), dim3(NT), 0, s, items,
                     chunks, count);
  TANQ_HIP(hipGetLastError());
}

void launch_batch(int k, tanq_prec p, const BatchItem* items, const BatchChunk* chunks, uint32_t* count,
                  hipStream_t s) {
  if (k == 2) {
    if (p == TANQ_F64) launch_batch_typed<double, 2>(items, chunks, count, s);
    else launch_batch_typed<float, 2>(items, chunks, count, s);
  } else if (k == 3) {
    if (p == TANQ_F64) launch_batch_typed<double, 3>(items, chunks, count, s);
    else launch_batch_typed<float, 3>(items, chunks, count, s);
  } else {
    fail(TANQ_E_ARG, "batched width must be 2 or 3");
  }
}

}  // namespace tanq
