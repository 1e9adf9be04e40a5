// Superoperator apply kernels of libtanq for gfx950 (CDNA4, wave64): the hot path.
//
// Applying a k-qubit superoperator S (4^k x 4^k complex) to vec(rho) in place is the batched
// GEMM [4^k x 4^k] x [4^k x 4^(n-k)] whose columns are the groups of amplitudes that differ
// only in the 2k target bits (Sec. 3.1, the "im2col" view; Sec. 3.2 maps the 2-qubit case
// onto FP64 tensor cores).
//
// Tiles.  A workgroup owns tiles of 2^V elements: the 2k target bits plus the lowest free
// bits, so every group lies in one tile and the tile is a union of contiguous runs of at least
// 2^(V-2k) elements.  Tiles move with 16-byte per-lane accesses (coalesced) through LDS; the
// grid is persistent; the next tile is prefetched into registers while the current one is
// multiplied, and the loop is rotated so that waiting for that prefetch never waits for the
// previous tile's stores.  Barriers fence LDS only, so global loads and stores stay in flight
// across them.  A second staging mode (apply_dma_kernel) streams the next tile straight into
// a second LDS buffer with global-to-LDS loads instead of through registers.
//
// LDS swizzle.  Element e of a tile lives at LDS element e ^ X(e), where X copies up to four
// group-index bits that lie above the 256-byte bank window into target-bit positions inside
// it.  The 16 groups of an MFMA column block then fall on distinct banks for every qubit
// placement, and X is constant on each 256-byte window, so the 16-byte load and store phases
// stay conflict-free.
//
// k = 2 (HBM-bound): real-block form.  Interleaved data is a real vector of length 32 and S the
// 32 x 32 real matrix [[Sr, -Si], [Si, Sr]] (interleaved); each wave owns 16-group column
// blocks and all of S: 2 m-tiles x 8 k-steps of 16x16x4 MFMA per block.
// k = 3 (MFMA-bound): 3M form, P1 = Sr xr, P2 = Si xi, P3 = (Sr + Si)(xr + xi),
// Re = P1 - P2, Im = P3 - P1 - P2: three real 64 x 64 products instead of four.  Each wave holds
// one 16-row m-tile of (Sr, Si, Sr + Si) and a share of the tile's column blocks; a barrier
// separates the reads of the tile from the in-place LDS writes.
// k = 1 (the paper's C1, kept off the matrix units as in the paper): VALU over the s_i map.
#include <atomic>
#include <cstring>
#include <type_traits>

#include "tile.hpp"

namespace tanq {

// One kernel for k = 2 and k = 3 on a single state: persistent grid over tiles, the next tile
// prefetched into registers while the current one is multiplied in LDS, and the loop rotated
// so that waiting for that prefetch leaves the previous tile's stores in flight (the wait
// only drains the vector-memory counter down to the number of outstanding stores).
template <typename T, int K, int VMAX, int NT, bool FULL>
__global__ __launch_bounds__(NT) void apply_tiles_kernel(T* __restrict__ rho, const T* __restrict__ frag,
                                                         const ApplyGeom g) {
  using IO = TileIo<T, VMAX, NT>;
  using Op = std::conditional_t<K == 2, Op2<T, VMAX, NT>, Op3<T, VMAX, NT>>;
  using c2 = typename Mfma<T>::c2;

  __shared__ u32x4 lds[IO::SLOTS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  IO io;
  io.init(g, tid);
  Op op;
  if constexpr (K == 2)
    op.load(frag, lane);
  else
    op.load(frag, lane, wave);
  op.prepare(g, lane, wave);

  uint64_t tile = xcd_first_tile();
  if (tile >= g.ntiles) return;  // uniform per workgroup
  uint64_t cur = tile_base(g, tile);
  u32x4 buf[IO::ITERS];
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) buf[it] = *reinterpret_cast<const u32x4*>(rho + 2 * (cur + io.off[it]));
#pragma unroll
  for (int it = 0; it < IO::ITERS; ++it)
    if (io.template has<FULL>(it, tid)) lds[io.lslot[it]] = buf[it];
  lds_barrier();

  for (;;) {
    const uint64_t next = tile + gridDim.x;
    const bool more = next < g.ntiles;
    uint64_t nbase = 0;
    if (more) {
      nbase = tile_base(g, next);
#pragma unroll
      for (int it = 0; it < IO::ITERS; ++it)
        if (io.template has<FULL>(it, tid)) buf[it] = *reinterpret_cast<const u32x4*>(rho + 2 * (nbase + io.off[it]));
    }

    if constexpr (K == 2)
      op.template compute<FULL>(reinterpret_cast<T*>(lds), g, lane, wave);
    else
      op.template compute<FULL>(reinterpret_cast<c2*>(lds), g, lane, wave);
    lds_barrier();

#pragma unroll
    for (int it = 0; it < IO::ITERS; ++it)
      if (io.template has<FULL>(it, tid)) *reinterpret_cast<u32x4*>(rho + 2 * (cur + io.off[it])) = lds[io.lslot[it]];
    if (!more) break;
    lds_barrier();  // every store-phase LDS read is done before the next tile lands
#pragma unroll
    for (int it = 0; it < IO::ITERS; ++it)
      if (io.template has<FULL>(it, tid)) lds[io.lslot[it]] = buf[it];
    lds_barrier();
    tile = next;
    cur = nbase;
  }
}

// The same multiplication with the tiles staged by direct global-to-LDS loads into two LDS
// buffers: the next tile streams into one buffer while the current one is multiplied in the
// other, without passing through registers (which frees the prefetch registers and keeps the
// HBM reads in flight for the whole multiplication).  Full tiles only.  The waits count this
// wave's vector-memory operations in issue order: previous tile's stores, then the next
// tile's loads, are allowed to remain outstanding.
template <typename T, int K, int VMAX, int NT>
__global__ __launch_bounds__(NT) void apply_dma_kernel(T* __restrict__ rho, const T* __restrict__ frag,
                                                       const ApplyGeom g) {
  using IO = TileDma<T, VMAX, NT>;
  using Op = std::conditional_t<K == 2, Op2<T, VMAX, NT>, Op3<T, VMAX, NT>>;
  using c2 = typename Mfma<T>::c2;

  __shared__ u32x4 lds[2][IO::SLOTS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  IO io;
  io.init(g, tid);
  Op op;
  if constexpr (K == 2)
    op.load(frag, lane);
  else
    op.load(frag, lane, wave);
  op.prepare(g, lane, wave);

  uint64_t tile = xcd_first_tile();
  if (tile >= g.ntiles) return;  // uniform per workgroup
  uint64_t cur = tile_base(g, tile);
  io.load(rho, cur, lds[0], tid, wave);
  int b = 0;
  bool first = true;
  for (;;) {
    const uint64_t next = tile + gridDim.x;
    const bool more = next < g.ntiles;
    uint64_t nbase = 0;
    if (more) {
      nbase = tile_base(g, next);
      io.load(rho, nbase, lds[b ^ 1], tid, wave);
      if (first)
        vm_wait<IO::ITERS>();
      else
        vm_wait<2 * IO::ITERS>();
    } else {
      if (first)
        vm_wait<0>();
      else
        vm_wait<IO::ITERS>();
    }
    raw_barrier();  // this tile is in LDS for every wave

    if constexpr (K == 2)
      op.template compute<true, true>(reinterpret_cast<T*>(lds[b]), g, lane, wave);
    else
      op.template compute<true, true>(reinterpret_cast<c2*>(lds[b]), g, lane, wave);
    raw_barrier();

    io.store(rho, cur, lds[b], tid);
    if (!more) break;
    raw_barrier();  // every wave's reads of buffer b are done before it is refilled
    tile = next;
    cur = nbase;
    b ^= 1;
    first = false;
  }
}

// The direct-staging instances of the variant table, instantiated explicitly (implicit
// instantiation through the launch table did not emit every host-side kernel handle).
#define TANQ_DMA_INSTANCE(T, K, V, NT) \
  template __global__ void apply_dma_kernel<T, K, V, NT>(T*, const T*, const ApplyGeom);
TANQ_DMA_INSTANCE(double, 2, 11, 256)
TANQ_DMA_INSTANCE(double, 2, 12, 512)
TANQ_DMA_INSTANCE(double, 3, 12, 512)
TANQ_DMA_INSTANCE(double, 3, 11, 512)
TANQ_DMA_INSTANCE(double, 3, 10, 256)
TANQ_DMA_INSTANCE(float, 2, 12, 256)
TANQ_DMA_INSTANCE(float, 2, 13, 512)
TANQ_DMA_INSTANCE(float, 3, 12, 256)
TANQ_DMA_INSTANCE(float, 3, 11, 256)
#undef TANQ_DMA_INSTANCE

// ------------------------------------------------------------------------------------
// C1 apply (k = 1): VALU, one group of four amplitudes per thread
// ------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void apply_c1_kernel(T* __restrict__ rho, const double* __restrict__ S,
                                                      const C1Geom g) {
  using c2 = typename Mfma<T>::c2;
  T sr[16], si[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    sr[i] = (T)S[2 * i];
    si[i] = (T)S[2 * i + 1];
  }
  const int q = g.q, n = g.n;
  const uint64_t lowmask = (1ull << q) - 1ull;
  const uint64_t midmask = (1ull << (n - 1)) - 1ull;
  const uint64_t dr = 1ull << q, dc = 1ull << (q + n);
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < g.ngroups; i += (uint64_t)gridDim.x * 256u) {
    // s_i of Sec. 3.1: deposit i into every bit except q and q + n
    const uint64_t hi = i >> q;
    const uint64_t s = ((hi >> (n - 1)) << (q + n + 1)) | ((hi & midmask) << (q + 1)) | (i & lowmask);
    const uint64_t idx[4] = {s, s + dr, s + dc, s + dr + dc};
    c2 x[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = *reinterpret_cast<const c2*>(rho + 2 * idx[a]);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T yr = 0, yi = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        yr += sr[4 * a + b] * x[b][0] - si[4 * a + b] * x[b][1];
        yi += sr[4 * a + b] * x[b][1] + si[4 * a + b] * x[b][0];
      }
      *reinterpret_cast<c2*>(rho + 2 * idx[a]) = c2{yr, yi};
    }
  }
}

// ------------------------------------------------------------------------------------
// packing of FP64 superoperators into the kernels' A-operand lane layouts
// ------------------------------------------------------------------------------------

// k = 2, real block: R[m'][k'] for m' = 2a + cm, k' = 2b + ck is
//   (cm, ck) = (0,0): Re S[a][b]   (0,1): -Im S[a][b]   (1,0): Im S[a][b]   (1,1): Re S[a][b]
// stored as P[(mt * 8 + ks) * 64 + lane] = R[16 mt + lane % 16][4 ks + lane / 16].
// k = 3, 3M: P[((mt * 16 + ks) * 3 + c) * 64 + lane] = C_c[16 mt + lane % 16][4 ks + lane / 16]
//   with C_0 = Re S, C_1 = Im S, C_2 = Re S + Im S (summed in FP64, rounded once).
// k = 1: the FP64 superoperator itself (32 doubles), for both precisions.
template <typename T>
__device__ void pack_block(int k, const double* __restrict__ S, unsigned char* __restrict__ out) {
  if (k == 1) {
    double* P = reinterpret_cast<double*>(out);
    for (int e = threadIdx.x; e < 32; e += blockDim.x) P[e] = S[e];
  } else if (k == 2) {
    T* P = reinterpret_cast<T*>(out);
    for (int e = threadIdx.x; e < 2 * 8 * 64; e += blockDim.x) {
      const int lane = e & 63, rest = e >> 6;
      const int ks = rest % 8, mt = rest / 8;
      const int mrow = 16 * mt + (lane & 15), kcol = 4 * ks + (lane >> 4);
      const int a = mrow >> 1, cm = mrow & 1, b = kcol >> 1, ck = kcol & 1;
      const double re = S[2 * (a * 16 + b)], im = S[2 * (a * 16 + b) + 1];
      P[e] = (T)((cm == ck) ? re : (cm == 0 ? -im : im));
    }
  } else {
    T* P = reinterpret_cast<T*>(out);
    for (int e = threadIdx.x; e < 4 * 16 * 3 * 64; e += blockDim.x) {
      const int lane = e & 63, rest = e >> 6;
      const int c = rest % 3, ks = (rest / 3) % 16, mt = rest / 48;
      const int a = 16 * mt + (lane & 15), b = 4 * ks + (lane >> 4);
      const double re = S[2 * (a * 64 + b)], im = S[2 * (a * 64 + b) + 1];
      P[e] = (T)(c == 0 ? re : (c == 1 ? im : re + im));
    }
  }
}

template <typename T>
__global__ void pack_kernel(const FuseBlockDev* __restrict__ blocks, const double* __restrict__ raw,
                            unsigned char* __restrict__ packed) {
  const FuseBlockDev blk = blocks[blockIdx.x];
  pack_block<T>(blk.k, raw + 2 * blk.out_off, packed + blk.pack_off);
}

template <typename T>
__global__ void pack_one_kernel(int k, const double* __restrict__ raw, unsigned char* __restrict__ packed) {
  pack_block<T>(k, raw, packed);
}

// ------------------------------------------------------------------------------------
// host side: geometry, variants, launches
// ------------------------------------------------------------------------------------

static int cu_count() {
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  static thread_local int cached_dev = -1, cached = 0;
  if (cached_dev != dev) {
    hipDeviceProp_t prop;
    TANQ_HIP(hipGetDeviceProperties(&prop, dev));
    cached = prop.multiProcessorCount;
    cached_dev = dev;
  }
  return cached;
}

int device_cu_count() { return cu_count(); }

ApplyGeom make_apply_geom(int n, int k, const int* q, int vbits, tanq_prec p) {
  ApplyGeom g;
  std::memset(&g, 0, sizeof(g));
  const int nb = 2 * n;
  const int V = vbits < nb ? vbits : nb;
  // target bits in local-index order: bit t <-> row bit q_t, bit k + t <-> column bit q_t + n
  int tgt[6];
  for (int t = 0; t < k; ++t) {
    tgt[t] = q[t];
    tgt[k + t] = q[t] + n;
  }
  uint64_t vmask = 0;
  for (int t = 0; t < 2 * k; ++t) vmask |= 1ull << tgt[t];
  int need = V - 2 * k;
  for (int b = 0; b < nb && need > 0; ++b)
    if (!((vmask >> b) & 1ull)) {
      vmask |= 1ull << b;
      --need;
    }
  int cnt = 0;
  for (int b = 0; b < nb; ++b)
    if ((vmask >> b) & 1ull) g.vpos[cnt++] = (uint8_t)b;
  g.V = V;
  int tpos[6] = {0, 0, 0, 0, 0, 0};
  uint32_t tmask_local = 0;
  for (int t = 0; t < 2 * k; ++t)
    for (int b = 0; b < V; ++b)
      if (g.vpos[b] == tgt[t]) {
        tpos[t] = b;
        tmask_local |= 1u << b;
      }
  g.free_mask = ((1u << V) - 1u) & ~tmask_local;
  const int D = 1 << (2 * k);
  for (int l = 0; l < D; ++l) {
    uint32_t r = 0;
    for (int t = 0; t < 2 * k; ++t)
      if ((l >> t) & 1) r |= 1u << tpos[t];
    g.tj[l] = r;
  }
  g.G = 1 << (V - 2 * k);
  // LDS swizzle: the 256-byte bank window holds 16 (FP64) or 32 (FP32) elements; FP32 keeps
  // element bit 0 (the two elements of a 16-byte slot stay together).
  {
    const int w = (p == TANQ_F64) ? 4 : 5;
    const int lo = (p == TANQ_F64) ? 0 : 1;
    int c = 0;
    for (int b = 0; b < w && b < V; ++b)
      if ((g.free_mask >> b) & 1u) ++c;
    int want = 4 - c;
    uint32_t xd = 0, xs = 0;
    int nd = 0;
    for (int b = lo; b < w && b < V && nd < want; ++b)
      if (!((g.free_mask >> b) & 1u)) {
        xd |= 1u << b;
        ++nd;
      }
    int ns = 0;
    for (int b = w; b < V && ns < nd; ++b)
      if ((g.free_mask >> b) & 1u) {
        xs |= 1u << b;
        ++ns;
      }
    // equal counts: drop surplus destination bits
    while (nd > ns) {
      xd &= ~(1u << (31 - __builtin_clz(xd)));
      --nd;
    }
    // source bits lie above the window and destination bits inside it, so the map is an
    // involution (the direct-to-LDS staging relies on that)
    if (xs & xd) fail(TANQ_E_STATE, "LDS swizzle masks overlap");
    g.xsrc = xs;
    g.xdst = xd;
  }
  // runs of fixed bits
  int src = 0, nr = 0;
  for (int b = 0; b < nb;) {
    if ((vmask >> b) & 1ull) {
      ++b;
      continue;
    }
    int e = b;
    while (e < nb && !((vmask >> e) & 1ull)) ++e;
    g.run_src[nr] = (uint8_t)src;
    g.run_len[nr] = (uint8_t)(e - b);
    g.run_dst[nr] = (uint8_t)b;
    src += e - b;
    ++nr;
    b = e;
  }
  g.nruns = nr;
  g.ntiles = 1ull << (nb - V);
  return g;
}

template <typename KernelT>
static uint64_t persistent_cap(KernelT kernel, int threads) {
  int per_cu = 0;
  TANQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
  if (per_cu < 1) per_cu = 1;
  return (uint64_t)cu_count() * (uint64_t)per_cu;
}

template <typename T, int K, int VMAX, int NT, bool FULL>
static void launch_tiles(const ApplyGeom& g, void* rho, const void* frag, hipStream_t s) {
  auto kern = apply_tiles_kernel<T, K, VMAX, NT, FULL>;
  static thread_local int cap_dev = -1;
  static thread_local uint64_t cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (cap_dev != dev) {
    cap = persistent_cap(kern, NT);
    cap_dev = dev;
  }
  const uint64_t grid = g.ntiles < cap ? g.ntiles : cap;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, (T*)rho, (const T*)frag, g);
  TANQ_HIP(hipGetLastError());
}

template <typename T, int K, int VMAX, int NT>
static void launch_dma(const ApplyGeom& g, void* rho, const void* frag, hipStream_t s) {
  auto kern = apply_dma_kernel<T, K, VMAX, NT>;
  static thread_local int cap_dev = -1;
  static thread_local uint64_t cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (cap_dev != dev) {
    cap = persistent_cap(kern, NT);
    cap_dev = dev;
  }
  const uint64_t grid = g.ntiles < cap ? g.ntiles : cap;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, (T*)rho, (const T*)frag, g);
  TANQ_HIP(hipGetLastError());
}

// STAGING 0: register prefetch (apply_tiles_kernel); 1: direct global-to-LDS loads into two
// LDS buffers (apply_dma_kernel) for full tiles, the register kernel for partial ones.
template <typename T, int K, int VMAX, int NT, int STAGING>
static void launch_variant(void* rho, int n, const int* qubits, const void* frag, hipStream_t s) {
  const ApplyGeom g = make_apply_geom(n, K, qubits, VMAX, sizeof(T) == 8 ? TANQ_F64 : TANQ_F32);
  if (g.V == VMAX) {
    if constexpr (STAGING == 1)
      launch_dma<T, K, VMAX, NT>(g, rho, frag, s);
    else
      launch_tiles<T, K, VMAX, NT, true>(g, rho, frag, s);
  } else {
    launch_tiles<T, K, VMAX, NT, false>(g, rho, frag, s);
  }
}

typedef void (*apply_fn)(void*, int, const int*, const void*, hipStream_t);

struct VariantEntry {
  int k;
  tanq_prec p;
  int tile_bits;
  int threads;
  int staging;
  apply_fn fn;
};

// Apply-kernel variants (tile bits x workgroup size); the first of each (k, precision) is the
// default until the autotuner or the caller selects another.
static const VariantEntry kVariants[] = {
    {2, TANQ_F64, 10, 256, 0, launch_variant<double, 2, 10, 256, 0>},
    {2, TANQ_F64, 11, 256, 0, launch_variant<double, 2, 11, 256, 0>},
    {2, TANQ_F64, 11, 512, 0, launch_variant<double, 2, 11, 512, 0>},
    {2, TANQ_F64, 12, 512, 0, launch_variant<double, 2, 12, 512, 0>},
    {2, TANQ_F64, 11, 256, 1, launch_variant<double, 2, 11, 256, 1>},
    {2, TANQ_F64, 12, 512, 1, launch_variant<double, 2, 12, 512, 1>},
    {2, TANQ_F32, 11, 256, 0, launch_variant<float, 2, 11, 256, 0>},
    {2, TANQ_F32, 12, 256, 0, launch_variant<float, 2, 12, 256, 0>},
    {2, TANQ_F32, 12, 512, 0, launch_variant<float, 2, 12, 512, 0>},
    {2, TANQ_F32, 13, 512, 0, launch_variant<float, 2, 13, 512, 0>},
    {2, TANQ_F32, 12, 256, 1, launch_variant<float, 2, 12, 256, 1>},
    {2, TANQ_F32, 13, 512, 1, launch_variant<float, 2, 13, 512, 1>},
    {3, TANQ_F64, 12, 512, 0, launch_variant<double, 3, 12, 512, 0>},
    {3, TANQ_F64, 11, 256, 0, launch_variant<double, 3, 11, 256, 0>},
    {3, TANQ_F64, 11, 512, 0, launch_variant<double, 3, 11, 512, 0>},
    {3, TANQ_F64, 10, 256, 0, launch_variant<double, 3, 10, 256, 0>},
    {3, TANQ_F64, 12, 512, 1, launch_variant<double, 3, 12, 512, 1>},
    {3, TANQ_F64, 11, 512, 1, launch_variant<double, 3, 11, 512, 1>},
    {3, TANQ_F64, 10, 256, 1, launch_variant<double, 3, 10, 256, 1>},
    {3, TANQ_F32, 12, 512, 0, launch_variant<float, 3, 12, 512, 0>},
    {3, TANQ_F32, 12, 256, 0, launch_variant<float, 3, 12, 256, 0>},
    {3, TANQ_F32, 13, 512, 0, launch_variant<float, 3, 13, 512, 0>},
    {3, TANQ_F32, 11, 256, 0, launch_variant<float, 3, 11, 256, 0>},
    {3, TANQ_F32, 12, 256, 1, launch_variant<float, 3, 12, 256, 1>},
    {3, TANQ_F32, 11, 256, 1, launch_variant<float, 3, 11, 256, 1>},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

// Process-wide variant per (k, precision), as an index among that pair's variants, and the
// autotuned variant per (n, k, precision) (-1: none), which takes precedence for that n.
static std::atomic<int> g_selected[4][2];
static std::atomic<int> g_tuned[kTunedMaxN + 1][2][4];

static struct VariantTablesInit {
  VariantTablesInit() {
    for (auto& a : g_selected)
      for (auto& b : a) b.store(0);
    for (auto& a : g_tuned)
      for (auto& b : a)
        for (auto& c : b) c.store(-1);
  }
} g_variant_tables_init;

static inline int pidx(tanq_prec p) { return p == TANQ_F64 ? 0 : 1; }

static int variant_global_index(int k, tanq_prec p, int local) {
  int c = 0;
  for (int i = 0; i < kNumVariants; ++i)
    if (kVariants[i].k == k && kVariants[i].p == p) {
      if (c == local) return i;
      ++c;
    }
  return -1;
}

int variant_count(int k, tanq_prec p) {
  int c = 0;
  for (int i = 0; i < kNumVariants; ++i)
    if (kVariants[i].k == k && kVariants[i].p == p) ++c;
  return c;
}

bool variant_describe(int k, tanq_prec p, int local, int* tile_bits, int* threads, int* staging) {
  const int gi = variant_global_index(k, p, local);
  if (gi < 0) return false;
  if (tile_bits) *tile_bits = kVariants[gi].tile_bits;
  if (threads) *threads = kVariants[gi].threads;
  if (staging) *staging = kVariants[gi].staging;
  return true;
}

int variant_find(int k, tanq_prec p, int tile_bits, int threads, int staging) {
  int c = 0;
  for (int i = 0; i < kNumVariants; ++i)
    if (kVariants[i].k == k && kVariants[i].p == p) {
      if (kVariants[i].tile_bits == tile_bits && kVariants[i].threads == threads && kVariants[i].staging == staging)
        return c;
      ++c;
    }
  return -1;
}

bool variant_select(int k, tanq_prec p, int local) {
  if (variant_global_index(k, p, local) < 0) return false;
  g_selected[k][pidx(p)].store(local);
  for (int n = 0; n <= kTunedMaxN; ++n) g_tuned[n][pidx(p)][k].store(-1);  // an explicit choice wins
  return true;
}

int variant_selected(int k, tanq_prec p) { return g_selected[k][pidx(p)].load(); }

bool variant_tune(int n, int k, tanq_prec p, int local) {
  if (n < 1 || n > kTunedMaxN || (local >= 0 && variant_global_index(k, p, local) < 0)) return false;
  g_tuned[n][pidx(p)][k].store(local);
  return true;
}

int variant_tuned(int n, int k, tanq_prec p) {
  return (n >= 1 && n <= kTunedMaxN) ? g_tuned[n][pidx(p)][k].load() : -1;
}

int variant_for(int n, int k, tanq_prec p) {
  const int t = variant_tuned(n, k, p);
  return t >= 0 ? t : variant_selected(k, p);
}

void launch_apply_variant(void* rho, int n, tanq_prec p, int k, int local, const int* qubits, const void* packed,
                          hipStream_t s) {
  const int gi = variant_global_index(k, p, local);
  if (gi < 0) fail(TANQ_E_ARG, "no such apply variant");
  kVariants[gi].fn(rho, n, qubits, packed, s);
}

void launch_apply(void* rho, int n, tanq_prec p, int k, const int* qubits, const void* packed, hipStream_t s) {
  if (k == 1) {
    C1Geom g{1ull << (2 * (n - 1)), qubits[0], n};
    uint64_t blocks = (g.ngroups + 255) / 256;
    const uint64_t cap = (uint64_t)cu_count() * 32;
    if (blocks > cap) blocks = cap;
    if (p == TANQ_F64)
      hipLaunchKernelGGL(apply_c1_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)rho,
                         (const double*)packed, g);
    else
      hipLaunchKernelGGL(apply_c1_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)rho,
                         (const double*)packed, g);
    TANQ_HIP(hipGetLastError());
    return;
  }
  if (k != 2 && k != 3) fail(TANQ_E_ARG, "superoperator width must be 1, 2 or 3");
  launch_apply_variant(rho, n, p, k, variant_for(n, k, p), qubits, packed, s);
}

void launch_pack(const FuseBlockDev* blocks, int nblocks, const double* raw, void* packed, tanq_prec p,
                 hipStream_t s) {
  if (nblocks <= 0) return;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(pack_kernel<double>, dim3(nblocks), dim3(256), 0, s, blocks, raw, (unsigned char*)packed);
  else
    hipLaunchKernelGGL(pack_kernel<float>, dim3(nblocks), dim3(256), 0, s, blocks, raw, (unsigned char*)packed);
  TANQ_HIP(hipGetLastError());
}

void launch_pack_one(int k, const double* raw, void* packed, tanq_prec p, hipStream_t s) {
  if (p == TANQ_F64)
    hipLaunchKernelGGL(pack_one_kernel<double>, dim3(1), dim3(256), 0, s, k, raw, (unsigned char*)packed);
  else
    hipLaunchKernelGGL(pack_one_kernel<float>, dim3(1), dim3(256), 0, s, k, raw, (unsigned char*)packed);
  TANQ_HIP(hipGetLastError());
}

}  // namespace tanq
