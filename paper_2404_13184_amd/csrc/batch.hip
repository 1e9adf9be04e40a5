// Batched superoperator apply for the serving loop (gfx950): one launch applies the next fused
// superoperator of every active request to that request's own vec(rho).  The work is a list of
// chunks (request item, range of tiles); a persistent grid walks the list, stages each item's
// tile geometry in LDS and runs the same in-place tile multiplication as the single-state
// kernels (tile.hpp).  States of different requests are disjoint, so the chunks of one launch
// are independent; successive launches are ordered on the stream.  The number of chunks is read
// from device memory, which lets a fixed launch be captured in a graph and replayed.
#include <type_traits>

#include "tile.hpp"

namespace tanq {

template <typename T, int K, int VMAX, int NT>
__global__ __launch_bounds__(NT) void batch_apply_kernel(const BatchItem* __restrict__ items,
                                                         const BatchChunk* __restrict__ chunks,
                                                         const uint32_t* __restrict__ count) {
  using IO = TileIo<T, VMAX, NT, false>;
  using Op = std::conditional_t<K == 2, Op2<T, NT>, Op3<T, VMAX, NT>>;
  using c2 = typename Mfma<T>::c2;
  static_assert(sizeof(ApplyGeom) % 4 == 0, "geometry copied as dwords");

  __shared__ u32x4 lds[IO::SLOTS];
  __shared__ ApplyGeom sg;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nch = *count;

  uint32_t cur = 0xffffffffu;
  IO io;
  Op op;
  T* rho = nullptr;
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const BatchChunk ch = chunks[c];
    if (ch.item != cur) {
      __syncthreads();  // the previous item's geometry is no longer read
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&items[ch.item].g);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sg);
      for (int i = tid; i < (int)(sizeof(ApplyGeom) / 4); i += NT) dst[i] = src[i];
      __syncthreads();
      rho = reinterpret_cast<T*>(items[ch.item].rho);
      const T* frag = reinterpret_cast<const T*>(items[ch.item].frag);
      io.init(sg, tid);
      if constexpr (K == 2)
        op.load(frag, lane);
      else
        op.load(frag, lane, wave);
      cur = ch.item;
    }
    for (uint32_t t = ch.tile_begin; t < ch.tile_end; ++t) {
      const uint64_t base = tile_base(sg, t);
      u32x4 buf[IO::ITERS];
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.has(it, tid)) buf[it] = *reinterpret_cast<const u32x4*>(rho + 2 * (base + io.off[it]));
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.has(it, tid)) lds[io.lslot[it]] = buf[it];
      __syncthreads();
      if constexpr (K == 2)
        op.compute(reinterpret_cast<T*>(lds), sg, lane, wave);
      else
        op.compute(reinterpret_cast<c2*>(lds), sg, lane, wave);
      __syncthreads();
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.has(it, tid)) *reinterpret_cast<u32x4*>(rho + 2 * (base + io.off[it])) = lds[io.lslot[it]];
      __syncthreads();
    }
  }
}

// Shapes: 16 KiB tiles for k = 2 (2^10 FP64 / 2^11 FP32 elements); k = 3 uses 2^11 (FP64) and
// 2^12 (FP32) elements, which keeps the FP64 instance free of register spills.
template <typename T, int K>
struct BatchShape;
template <>
struct BatchShape<double, 2> { static constexpr int V = 10, NT = 256; };
template <>
struct BatchShape<float, 2> { static constexpr int V = 11, NT = 256; };
template <>
struct BatchShape<double, 3> { static constexpr int V = 11, NT = 512; };
template <>
struct BatchShape<float, 3> { static constexpr int V = 12, NT = 512; };

int batch_tile_bits(int k, tanq_prec p) {
  if (k == 2) return p == TANQ_F64 ? BatchShape<double, 2>::V : BatchShape<float, 2>::V;
  return p == TANQ_F64 ? BatchShape<double, 3>::V : BatchShape<float, 3>::V;
}

template <typename T, int K>
static void launch_batch_typed(const BatchItem* items, const BatchChunk* chunks, const uint32_t* count,
                               hipStream_t s) {
  constexpr int V = BatchShape<T, K>::V, NT = BatchShape<T, K>::NT;
  auto kern = batch_apply_kernel<T, K, V, NT>;
  static thread_local int cap_dev = -1;
  static thread_local unsigned cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (cap_dev != dev) {
    int per_cu = 0;
    TANQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0));
    cap = (unsigned)(device_cu_count() * (per_cu < 1 ? 1 : per_cu));
    cap_dev = dev;
  }
  hipLaunchKernelGGL(kern, dim3(cap), dim3(NT), 0, s, items, chunks, count);
  TANQ_HIP(hipGetLastError());
}

void launch_batch(int k, tanq_prec p, const BatchItem* items, const BatchChunk* chunks, const uint32_t* count,
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
