// Multi-superoperator passes (gfx950): several consecutive 2-qubit superoperators applied to
// each tile of vec(rho) while it sits in LDS, so the state crosses HBM once per pass instead of
// once per superoperator.
//
// A pass is a run of fused 2-qubit blocks whose qubits together number at most V/2 (the tile
// holds the row and column bit of every one of them, plus the lowest other bits up to V).  For
// each superoperator of the pass the tile splits into 2^(V-4) groups of 16 elements, indexed by
// the tile bits that are not its targets, and every group is multiplied by the 16 x 16 complex
// superoperator as in the single-superoperator kernel (Sec. 3.1-3.2's batched GEMM), here in
// 3M form (three real MFMA products instead of the real-block form's four).  Superoperators
// follow one another in circuit order, separated by an LDS barrier, so the result is that of
// applying them one by one, up to the rounding of the two forms.
//
// LDS swizzle.  One LDS layout serves every superoperator of the pass, so the swizzle is a
// linear map over GF(2): element e lives at S(e) = e ^ X(e), where X XORs a W-bit value (W = 4
// for FP64, 5 for FP32: the 256-byte bank window) for each set bit of e above the window.  X
// depends only on bits above the window, so S permutes every window (the 16-byte load and store
// phases stay conflict-free) and S is its own inverse.  The host picks X so that, for every
// superoperator, the 16 groups an MFMA column block reads land on distinct banks (and, for FP32,
// also the two rows each lane pair covers); by linearity S(tile index of a target part + group
// part) = S(target part) ^ S(group part), so the target offsets are swizzled once on the host.
// In FP32 X never flips bit 0, so the two elements of a 16-byte slot stay in order.
//
// Kernels.  One workgroup per CU and two 64 KiB LDS tile buffers: the next tile streams into
// one with direct global-to-LDS loads while the current one is multiplied in the other and
// stored; each workgroup walks a contiguous range of tiles (pass_tiles).  FP32
// (apply_pass_ws_kernel): specialised waves, two producer waves issuing the loads and eight
// consumer waves that multiply, reading each superoperator's operands from LDS one
// superoperator ahead.  FP64 (apply_pass_kernel): eight waves that all multiply and each issue
// their share of the loads; two waves per SIMD leave enough registers to hold the operands of
// all (at most four) superoperators for the whole kernel.
#include "tile.hpp"

namespace tanq {

namespace {

template <typename T>
struct PassWin;
template <>
struct PassWin<double> { static constexpr int W = 4; };
template <>
struct PassWin<float> { static constexpr int W = 5; };

template <typename T>
__device__ inline uint32_t pass_swz(uint32_t e, const PassGeom& g) {
  uint32_t x = e;
#pragma unroll
  for (int b = PassWin<T>::W; b < 16; ++b)
    if ((e >> b) & 1u) x ^= g.xcol[b];
  return x;
}

__device__ inline uint64_t pass_tile_base(const PassGeom& g, uint64_t tile) {
  uint64_t b = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r)  // constant indices into the kernel-argument run table
    if (r < g.nruns) b |= ((tile >> g.run_src[r]) & ((1ull << g.run_len[r]) - 1ull)) << g.run_dst[r];
  return b;
}

}  // namespace

// Tiles of one workgroup of a pass launch: a contiguous range of ceil(ntiles / gridDim.x)
// tiles (the last ranges shorter or empty), so that consecutive tiles of a CU lie next to each
// other in vec(rho) instead of a grid apart.
struct PassTiles {
  uint64_t first, end;
};
__device__ inline PassTiles pass_tiles(uint64_t ntiles) {
  const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint64_t first = (uint64_t)blockIdx.x * per;
  return PassTiles{first, first + per < ntiles ? first + per : ntiles};
}

// Superoperators per pass: their 3M operands (768 elements each) are rebuilt in LDS beside the
// two 64 KiB tile buffers at the start of every launch.
template <typename T>
struct PassMax;
template <>
struct PassMax<double> { static constexpr int M = kPassMaxF64; };
template <>
struct PassMax<float> { static constexpr int M = kPassMaxF32; };

// Global offset of tile element e0 = S(first element of LDS slot p); the slot's EPS elements are
// consecutive in the tile and in vec(rho) (tile bit 0 is global bit 0, and this swizzle never
// flips bit 0 for FP32, so a slot's pair keeps its order).
template <typename T, int VMAX>
__device__ inline uint64_t pass_slot_off(uint32_t first, const PassGeom& g) {
  const uint32_t e = pass_swz<T>(first, g);
  uint64_t o = 0;
  for (int b = 0; b < VMAX; ++b) o |= (uint64_t)((e >> b) & 1u) << g.vpos[b];
  return o;
}

// Operands of a pass in LDS: each 2-qubit superoperator in 3M form, Sr, Si and Sr + Si as
// 4 k-steps x 3 x 64 lane fragments (lane l holds row l % 16, column 4 s + l / 16).
constexpr int kOp3M = 4 * 3 * 64;

// Build the 3M fragments of superoperator j from its real-block packing (the single-apply
// operand: the 32 x 32 real matrix [[Sr, -Si], [Si, Sr]] on interleaved indices, in MFMA lane
// order: element (R, C) at ((R / 16) * 8 + C / 4) * 64 + (C % 4) * 16 + R % 16).
template <typename T>
__device__ inline T pass_op3m(const T* __restrict__ rb, int r) {
  const int s3 = r / 192, t = (r / 64) % 3, lane = r % 64;
  const int a = lane % 16, b = 4 * s3 + lane / 16;  // complex row and column
  auto at = [&](int R, int C) { return rb[((R / 16) * 8 + C / 4) * 64 + (C % 4) * 16 + R % 16]; };
  const T sr = at(2 * a, 2 * b), si = at(2 * a + 1, 2 * b);
  return t == 0 ? sr : (t == 1 ? si : sr + si);
}

// One superoperator of a pass on the tile in ldsC, by consumer wave cw of NCW, in 3M form:
// P1 = Sr xr, P2 = Si xi, P3 = (Sr + Si)(xr + xi); Re = P1 - P2, Im = P3 - P1 - P2 -- three
// real 16 x 16 products per group instead of the real-block form's four.  A wave writes only
// the groups it read, so there is no barrier inside one superoperator.
//
// The work is split so that the matrix units of a SIMD stay busy across the barrier that
// separates superoperators: everything that does not depend on the tile (this lane's operand
// fragments and the swizzled tile index of its groups' rows) is read into registers while the
// previous superoperator is still multiplying (PassOps::load), every B operand of the
// superoperator is read from LDS right after the barrier (all column blocks at once, so the
// reads wait for nothing but their own latency), and the column blocks are multiplied one
// after the other, so the additions and LDS writes of one block's results overlap the next
// block's products.
template <typename T, int VMAX, int NCW>
struct PassOps {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using c2 = typename M::c2;
  static constexpr int G = 1 << (VMAX - 4);  // groups of one superoperator per tile
  static constexpr int NB = G / 16;          // column blocks (16 groups each)
  static constexpr int NBW = NB / NCW;       // column blocks per consumer wave
  static_assert(NB % NCW == 0, "every consumer wave gets the same number of column blocks");
  static constexpr int KS = 4;               // k-steps of 4 (16 complex columns)
  // Raw values read from LDS; nothing is computed from them until apply(), so reading them
  // never makes the wave wait.  st[l] = S(tile index of local index l); S and the deposit of l
  // into the tile are both linear over GF(2), so st[a ^ b] = st[a] ^ st[b].
  T ar[KS], ai[KS], as[KS];  // 3M fragments of this lane (row l % 16, column 4 s + l / 16)
  uint32_t gx[NBW];          // S(group part) of this lane's group in each of its column blocks
  uint32_t skk;              // st[kk], kk = lane / 16: this lane's B row within a k-step
  uint32_t srow;             // st[4 kk]: output row 4 kk of an FP32 accumulator (unused for FP64)
  u32x4 stk;                 // st[0], st[4], st[8], st[12]: the k-step row offsets
  u32x4 st0;                 // st[0..3]: FP32 accumulator rows 4 kk + r (unused for FP64)

  // stl: the superoperator's 16 offsets st[l] followed by st[0], st[4], st[8], st[12]
  __device__ inline void load(const T* __restrict__ op, const uint16_t* __restrict__ gxt, const uint32_t* stl, int cw,
                              int lane) {
    const int kk = lane >> 4;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      ar[s] = op[(s * 3 + 0) * 64 + lane];
      ai[s] = op[(s * 3 + 1) * 64 + lane];
      as[s] = op[(s * 3 + 2) * 64 + lane];
    }
#pragma unroll
    for (int i = 0; i < NBW; ++i) gx[i] = gxt[(cw + i * NCW) * 16 + (lane & 15)];
    skk = stl[kk];
    stk = *reinterpret_cast<const u32x4*>(stl + 16);
    if constexpr (!M::kRowsStrided) {
      srow = stl[4 * kk];
      st0 = *reinterpret_cast<const u32x4*>(stl);
    }
  }

  // B operands of every column block of this wave (issued right after the barrier)
  __device__ inline void read(const c2* ldsC, c2 (&v)[NBW][KS]) const {
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int s = 0; s < KS; ++s) v[i][s] = ldsC[(stk[s] ^ skk) ^ gx[i]];
  }

  struct Acc {
    acc_t p1, p2, p3;
  };

  // the three real products of column block i
  __device__ inline Acc products(const c2 (&v)[NBW][KS], int i) const {
    Acc a{acc_t{0, 0, 0, 0}, acc_t{0, 0, 0, 0}, acc_t{0, 0, 0, 0}};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const T br = v[i][s][0], bi = v[i][s][1];
      a.p1 = M::mma(ar[s], br, a.p1);
      a.p2 = M::mma(ai[s], bi, a.p2);
      a.p3 = M::mma(as[s], br + bi, a.p3);
    }
    return a;
  }

  // the 3M combination of block i written back in place; accumulator value r holds output row
  // kk + 4 r (FP64) or 4 kk + r (FP32)
  __device__ inline void write(c2* ldsC, const Acc& a, int i) const {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t e = M::kRowsStrided ? ((stk[r] ^ skk) ^ gx[i]) : ((st0[r] ^ srow) ^ gx[i]);
      ldsC[e] = c2{a.p1[r] - a.p2[r], a.p3[r] - a.p1[r] - a.p2[r]};
    }
  }
};

// Producer: stream one tile into buf with direct global-to-LDS loads (lane data lands at the
// wave's base + 16 * lane, so slot it * PT + tid receives the 16 bytes at offset off[it]).
// The loads and the consumers' stores are marked non-temporal (cache policy 2): a pass touches
// every element once, so nothing it moves is read again before the next pass.
template <typename T, int PITERS, int PT>
__device__ inline void pass_dma_tile(const T* rho, uint64_t base, const uint64_t (&off)[PITERS], u32x4* buf,
                                     int wave) {
#pragma unroll
  for (int it = 0; it < PITERS; ++it)
    __builtin_amdgcn_global_load_lds(rho + 2 * (base + off[it]), buf + it * PT + wave * 64, 16, 0, 2);
}

template <typename T, int VMAX, int NT, int NPW>
__global__ __launch_bounds__(NT) void apply_pass_ws_kernel(T* __restrict__ rho, const T* __restrict__ frags,
                                                           const PassGeom g) {
  constexpr int NCW = NT / 64 - NPW;
  constexpr int EPS = 16 / (2 * (int)sizeof(T));  // elements per 16-byte slot
  constexpr int SLOTS = (1 << VMAX) / EPS;
  constexpr int PT = NPW * 64, CT = NCW * 64;  // producer and consumer threads
  constexpr int PITERS = SLOTS / PT;           // loads per producer lane per tile
  constexpr int CITERS = SLOTS / CT;           // stores per consumer thread per tile
  static_assert(SLOTS % PT == 0 && SLOTS % CT == 0, "whole slots per thread");
  constexpr int G = 1 << (VMAX - 4);
  constexpr int MMAX = PassMax<T>::M;

  __shared__ u32x4 ldsA[SLOTS];
  __shared__ u32x4 ldsB[SLOTS];
  __shared__ T opl[MMAX][kOp3M];
  __shared__ uint16_t gxt[MMAX][G];
  // st[l] of every superoperator (16 words), then st[0], st[4], st[8], st[12]
  __shared__ __align__(16) uint32_t stl[MMAX][20];
  // global offset of the part it * CT of a consumer's store slot index, it < CITERS
  __shared__ uint64_t soff[CITERS];
  // base offset of the tile in each buffer, written by the producer with its loads: the
  // consumers take it from LDS rather than recomputing it from the run table (which the
  // compiler may read with vector loads, and waiting for those would wait for the stores)
  __shared__ uint64_t tbase[2];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  const PassTiles range = pass_tiles(g.ntiles);
  uint64_t tile = range.first;
  if (tile >= range.end) return;  // uniform per workgroup
  for (int idx = tid; idx < g.m * kOp3M; idx += NT)
    opl[idx / kOp3M][idx % kOp3M] = pass_op3m<T>(frags + g.op_off[idx / kOp3M], idx % kOp3M);
  if (tid < CITERS) soff[tid] = pass_slot_off<T, VMAX>((uint32_t)(tid * CT * EPS), g);
  for (int idx = tid; idx < g.m * 20; idx += NT) {
    const int j = idx / 20, l = idx % 20;
    stl[j][l] = g.stj[j][l < 16 ? l : 4 * (l - 16)];
  }
  for (int idx = tid; idx < g.m * G; idx += NT) {
    const int j = idx / G, gi = idx % G;
    gxt[j][gi] = (uint16_t)pass_swz<T>(pdep32((uint32_t)gi, g.free_mask[j]), g);
  }
  lds_barrier();  // operands and table in place before the roles split

  if (wave < NPW) {
    // ---------------- producer ----------------
    uint64_t off[PITERS];
#pragma unroll
    for (int it = 0; it < PITERS; ++it) off[it] = pass_slot_off<T, VMAX>((uint32_t)((it * PT + tid) * EPS), g);
    {
      const uint64_t base = pass_tile_base(g, tile);
      if (tid == 0) tbase[0] = base;
      pass_dma_tile<T, PITERS, PT>(rho, base, off, ldsA, wave);
    }
    vm_wait<0>();
    raw_barrier();  // B0: first tile ready
    for (int t = 0;; ++t) {
      const uint64_t next = tile + 1;
      const bool more = next < range.end;
      if (more) {
        // tbase[(t + 1) & 1] was last read before this tile's B0
        const uint64_t base = pass_tile_base(g, next);
        if (tid == 0) tbase[(t + 1) & 1] = base;
        pass_dma_tile<T, PITERS, PT>(rho, base, off, (t & 1) ? ldsA : ldsB, wave);
      }
      for (int j = 0; j <= g.m; ++j) raw_barrier();  // the m superoperators, then B_free
      if (!more) break;
      vm_wait<0>();
      raw_barrier();  // B0: next tile ready
      tile = next;
    }
  } else {
    // ---------------- consumers ----------------
    using Ops = PassOps<T, VMAX, NCW>;
    using c2 = typename Mfma<T>::c2;
    const int cw = wave - NPW;  // consumer wave 0..NCW-1
    const int ct = tid - PT;    // consumer thread 0..CT-1
    // global offset of the slots this thread stores: the slot index it * CT + ct splits into
    // disjoint bit fields and the offset is linear in them over GF(2) (swizzle and bit deposit
    // are), so offset = offset(ct part) ^ offset(it part), the latter the same for every thread
    const uint64_t off_ct = pass_slot_off<T, VMAX>((uint32_t)(ct * EPS), g);
    // two operand sets: superoperator j multiplies with ops[j & 1] while ops[(j + 1) & 1] is
    // filled for j + 1 (for superoperator 0 of the next tile after the last one)
    Ops ops[2];
    ops[0].load(opl[0], gxt[0], stl[0], cw, lane);
    raw_barrier();  // B0: first tile ready
    for (int t = 0;; ++t) {
      const uint64_t cur = tbase[t & 1];
      const uint64_t next = tile + 1;
      const bool more = next < range.end;
      u32x4* buf = (t & 1) ? ldsB : ldsA;
      c2* bufC = reinterpret_cast<c2*>(buf);
#pragma unroll
      for (int j = 0; j < MMAX; ++j) {
        if (j >= g.m) break;  // uniform
        c2 v[Ops::NBW][Ops::KS];
        typename Ops::Acc acc[2];
        const Ops& o = ops[j & 1];
        o.read(bufC, v);
        // LDS returns in order: the first column block's products are issued before the next
        // operands are requested (unconditionally, so the waits can count them: after the last
        // superoperator, superoperator 0 of the next tile), so they wait only for their B reads
        __builtin_amdgcn_sched_barrier(0);
        acc[0] = o.products(v, 0);
        __builtin_amdgcn_sched_barrier(0);
        {
          const int jn = (j + 1 < g.m) ? j + 1 : 0;
          ops[(j + 1) & 1].load(opl[jn], gxt[jn], stl[jn], cw, lane);
        }
        __builtin_amdgcn_sched_barrier(0);
        // block i's products, then block i - 1's results: the additions and LDS writes of one
        // block run while the matrix units work on the next
#pragma unroll
        for (int i = 1; i < Ops::NBW; ++i) {
          acc[i & 1] = o.products(v, i);
          o.write(bufC, acc[(i - 1) & 1], i - 1);
        }
        o.write(bufC, acc[(Ops::NBW - 1) & 1], Ops::NBW - 1);
        raw_barrier();  // the next superoperator (or the store) reads what other waves wrote
      }
      if (g.m & 1) ops[0] = ops[1];  // the last superoperator left superoperator 0 in ops[m & 1]
#pragma unroll
      for (int it = 0; it < CITERS; ++it)
        __builtin_nontemporal_store(buf[it * CT + ct], reinterpret_cast<u32x4*>(rho + 2 * (cur + (off_ct ^ soff[it]))));
      raw_barrier();  // B_free: this buffer is read out
      if (!more) break;
      raw_barrier();  // B0: next tile ready
      tile = next;
    }
  }
}

// Direct global-to-LDS load of 16 bytes per lane into the LDS slots starting at lds_base (the
// wave's base: lane l fills lds_base + 16 l), with the non-temporal policy.  Written as
// assembly because the compiler cannot tell this wave's two tile buffers apart: with the
// builtin it would wait for every such load before each LDS read of the other buffer, which
// removes the overlap of the next tile's loads with this tile's multiplication.  The
// instruction is the one the builtin emits: its only register operand is the address, read
// when it issues, and it has no register outputs (the data goes to LDS), so nothing the
// compiler allocates is written while it is in flight.  The compiler does not count it, so the
// kernel orders it itself: no LDS access touches the destination buffer until this wave has
// waited for its loads (vm_wait) and the workgroup has passed the barrier that publishes the
// tile, and no load is left in flight at the end of the kernel.
__device__ inline void pass_dma16(const void* gaddr, uint32_t lds_base) {
  // M0 holds the LDS address; one wait state between writing M0 and the load that reads it
  asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt" ::"v"(gaddr), "{m0}"(lds_base) : "memory");
}

__device__ inline uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// One tile of the consumer-only pass: the next tile's loads into `other`, the m superoperators
// on `buf` with every operand in registers (ops[j]), then the store of `buf`.
template <typename T, int VMAX, int NT, int MMAX, int ITERS, typename Ops>
__device__ inline void pass_cw_tile(T* __restrict__ rho, const Ops (&ops)[MMAX], int m, u32x4* buf, u32x4* other,
                                    uint64_t cur, uint64_t nbase, bool more, const uint64_t (&off)[ITERS], int tid,
                                    int wave) {
  using c2 = typename Mfma<T>::c2;
  c2* bufC = reinterpret_cast<c2*>(buf);
  if (more) {
    const uint32_t ob = lds_addr(other) + (uint32_t)wave * 1024u;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) pass_dma16(rho + 2 * (nbase + off[it]), ob + (uint32_t)(it * NT * 16));
  }
#pragma unroll
  for (int j = 0; j < MMAX; ++j) {
    if (j >= m) break;  // uniform
    c2 v[Ops::NBW][Ops::KS];
    typename Ops::Acc acc[2];
    const Ops& o = ops[j];
    o.read(bufC, v);
    __builtin_amdgcn_sched_barrier(0);
    acc[0] = o.products(v, 0);
#pragma unroll
    for (int i = 1; i < Ops::NBW; ++i) {
      acc[i & 1] = o.products(v, i);
      o.write(bufC, acc[(i - 1) & 1], i - 1);
    }
    o.write(bufC, acc[(Ops::NBW - 1) & 1], Ops::NBW - 1);
    raw_barrier();  // the next superoperator (or the store) reads what other waves wrote
  }
#pragma unroll
  for (int it = 0; it < ITERS; ++it)
    __builtin_nontemporal_store(buf[it * NT + tid], reinterpret_cast<u32x4*>(rho + 2 * (cur + off[it])));
}

// The same pass with consumer waves only: every wave multiplies, and each also issues its share
// of the next tile's direct global-to-LDS loads (the same slots it stores, so one offset table
// serves both).  Two waves per SIMD leave 256 registers per lane, enough to keep every
// superoperator's operands and offsets in registers for the whole kernel instead of reading
// them from LDS once per superoperator.  One barrier per tile fewer: after the store phase
// each wave waits only for its own loads of the next tile (the stores issued after them may
// still be in flight; the memory counter drains in issue order), and the barrier that
// publishes the next tile also frees the current buffer.
template <typename T, int VMAX, int NT>
__global__ __launch_bounds__(NT) void apply_pass_kernel(T* __restrict__ rho, const T* __restrict__ frags,
                                                        const PassGeom g) {
  constexpr int NW = NT / 64;
  constexpr int EPS = 16 / (2 * (int)sizeof(T));  // elements per 16-byte slot
  constexpr int SLOTS = (1 << VMAX) / EPS;
  constexpr int ITERS = SLOTS / NT;  // loads and stores per thread per tile
  static_assert(SLOTS % NT == 0, "whole slots per thread");
  static_assert(ITERS < 64, "a tile's loads fit the memory counter");
  constexpr int G = 1 << (VMAX - 4);
  constexpr int MMAX = PassMax<T>::M;
  using Ops = PassOps<T, VMAX, NW>;

  __shared__ u32x4 ldsA[SLOTS];
  __shared__ u32x4 ldsB[SLOTS];
  __shared__ T opl[MMAX][kOp3M];
  __shared__ uint16_t gxt[MMAX][G];
  __shared__ __align__(16) uint32_t stl[MMAX][20];
  __shared__ uint64_t soff[ITERS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  const PassTiles range = pass_tiles(g.ntiles);
  uint64_t tile = range.first;
  if (tile >= range.end) return;  // uniform per workgroup
  for (int idx = tid; idx < g.m * kOp3M; idx += NT)
    opl[idx / kOp3M][idx % kOp3M] = pass_op3m<T>(frags + g.op_off[idx / kOp3M], idx % kOp3M);
  if (tid < ITERS) soff[tid] = pass_slot_off<T, VMAX>((uint32_t)(tid * NT * EPS), g);
  for (int idx = tid; idx < g.m * 20; idx += NT) {
    const int j = idx / 20, l = idx % 20;
    stl[j][l] = g.stj[j][l < 16 ? l : 4 * (l - 16)];
  }
  for (int idx = tid; idx < g.m * G; idx += NT) {
    const int j = idx / G, gi = idx % G;
    gxt[j][gi] = (uint16_t)pass_swz<T>(pdep32((uint32_t)gi, g.free_mask[j]), g);
  }
  lds_barrier();

  static_assert(MMAX <= 4, "every superoperator's operands fit in registers");
  Ops ops[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j)
    if (j < g.m) ops[j].load(opl[j], gxt[j], stl[j], wave, lane);
  // global offset of slot it * NT + tid (linear over GF(2) in the slot index)
  uint64_t off[ITERS];
  {
    const uint64_t off_t = pass_slot_off<T, VMAX>((uint32_t)(tid * EPS), g);
#pragma unroll
    for (int it = 0; it < ITERS; ++it) off[it] = off_t ^ soff[it];
  }
  // The run table deposits the tile index into the global bits outside the tile, lowest first,
  // so the base of the next tile follows from the current one by an increment under that mask
  // (the bits outside it set so that the carry passes over them): three scalar operations per
  // tile instead of walking the run table at the start of every tile.
  uint64_t dmask = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if (r < g.nruns) dmask |= ((1ull << g.run_len[r]) - 1ull) << g.run_dst[r];
  uint64_t cur = pass_tile_base(g, tile);
  {
    const uint32_t ab = lds_addr(ldsA) + (uint32_t)wave * 1024u;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) pass_dma16(rho + 2 * (cur + off[it]), ab + (uint32_t)(it * NT * 16));
  }
  vm_wait<0>();
  raw_barrier();  // the first tile is in LDS
  for (int t = 0;; ++t) {
    const uint64_t next = tile + 1;
    const bool more = next < range.end;
    // the other buffer was read out before the barrier that published this tile
    const uint64_t nbase = more ? ((cur | ~dmask) + 1ull) & dmask : 0;
    if (t & 1)
      pass_cw_tile<T, VMAX, NT, MMAX, ITERS>(rho, ops, g.m, ldsB, ldsA, cur, nbase, more, off, tid, wave);
    else
      pass_cw_tile<T, VMAX, NT, MMAX, ITERS>(rho, ops, g.m, ldsA, ldsB, cur, nbase, more, off, tid, wave);
    if (!more) break;
    vm_wait<ITERS>();  // this wave's loads of the next tile (issued before its stores)
    raw_barrier();     // the next tile is in LDS; this buffer is read out
    tile = next;
    cur = nbase;
  }
}

// Tile sizes: 2^12 FP64 elements or 2^13 FP32 elements (64 KiB: six qubits, and one more bit
// in FP32).
template <typename T>
struct PassShape;
template <>
struct PassShape<double> { static constexpr int V = kPassTileBitsF64; };
template <>
struct PassShape<float> { static constexpr int V = kPassTileBitsF32; };

// Kernel and block size per precision: FP64 passes (at most four superoperators) run on
// consumer waves only, with every operand in registers; FP32 passes (up to six) keep the
// specialised waves, whose consumers read the operands one superoperator ahead (measured: the
// consumer-only form with operands read from LDS is 9% slower in FP32, the register-resident
// one 2-3% faster in FP64).
template <typename T>
struct PassKernel;
template <>
struct PassKernel<double> {
  static constexpr int NT = 512;
  static constexpr auto kern = apply_pass_kernel<double, kPassTileBitsF64, 512>;
};
template <>
struct PassKernel<float> {
  static constexpr int NT = 640;
  static constexpr auto kern = apply_pass_ws_kernel<float, kPassTileBitsF32, 640, 2>;
};

template <typename T>
static void launch_pass_typed(void* rho, const PassGeom& g, const void* frags, hipStream_t s) {
  constexpr int V = PassShape<T>::V, NT = PassKernel<T>::NT;
  if (g.V != V) fail(TANQ_E_STATE, "pass geometry built for another tile size");
  if (g.m < 1 || g.m > PassMax<T>::M) fail(TANQ_E_STATE, "pass longer than its operand buffers");
  auto kern = PassKernel<T>::kern;
  static thread_local int cap_dev = -1;
  static thread_local uint64_t cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (cap_dev != dev) {
    int per_cu = 0;
    TANQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0));
    cap = (uint64_t)device_cu_count() * (uint64_t)(per_cu < 1 ? 1 : per_cu);
    cap_dev = dev;
  }
  const uint64_t grid = g.ntiles < cap ? g.ntiles : cap;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, (T*)rho, (const T*)frags, g);
  TANQ_HIP(hipGetLastError());
}

void launch_pass(void* rho, tanq_prec p, const PassGeom& g, const void* frags, hipStream_t s) {
  if (p == TANQ_F64)
    launch_pass_typed<double>(rho, g, frags, s);
  else
    launch_pass_typed<float>(rho, g, frags, s);
}

}  // namespace tanq
