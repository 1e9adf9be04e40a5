// Device building blocks of the superoperator apply kernels (gfx950): MFMA lane layouts, the
// tile geometry helpers, the LDS swizzle and the in-place multiplication of one LDS tile for
// k = 2 (real-block form) and k = 3 (3M form).  Shared by the single-state kernels
// (apply.hip) and the batched serving kernel (batch.hip).
#pragma once

#include "internal.hpp"

namespace tanq {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Lane layouts (gfx950, checked with an in-bounds probe): for both 16x16x4 builtins lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16].  The four accumulator values of lane l
// are D[row][l % 16] with row = (l / 16) + 4 r for f64 and row = 4 (l / 16) + r for f32.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = f64x4;
  using c2 = f64x2;
  static constexpr bool kRowsStrided = true;  // row = (l/16) + 4r
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  using c2 = f32x2;
  static constexpr bool kRowsStrided = false;  // row = 4(l/16) + r
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Device memory reached through a pointer read from memory (a work-list entry): the compiler
// cannot tell which memory it points to and accesses it with flat instructions, which also
// count on the LDS counter, so every wait for an LDS read would also wait for them (the next
// tile's prefetch then no longer overlaps the multiplication).  Accesses through the returned
// pointer are global-memory instructions.
template <typename T>
__device__ inline __attribute__((address_space(1))) T* global_ptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ inline uint32_t pdep32(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  for (uint32_t m = mask; m; m &= m - 1) {
    if (x & 1u) r |= m & (0u - m);
    x >>= 1;
  }
  return r;
}

__device__ inline uint32_t pext32(uint32_t x, uint32_t mask) {
  uint32_t r = 0, bit = 1;
  for (uint32_t m = mask; m; m &= m - 1) {
    if (x & m & (0u - m)) r |= bit;
    bit <<= 1;
  }
  return r;
}

// LDS swizzle: element e of a tile lives at LDS element e ^ X(e), where X copies up to four
// group-index bits lying above the 256-byte bank window into target-bit positions inside it
// (masks xsrc, xdst from make_apply_geom).  The 16 groups of an MFMA column block then fall on
// distinct banks for every qubit placement, and X is constant on each 256-byte window, so the
// 16-byte load and store phases stay conflict-free.
template <typename G>
__device__ inline uint32_t swz(uint32_t e, const G& g) {
  return pdep32(pext32(e, g.xsrc), g.xdst);
}

// Global element offset and swizzled LDS slot of every 16-byte slot a thread moves; the same
// for every tile of one geometry.  has<true>: the tile has all 2^VMAX elements, so no
// per-slot guard (a guard around each access makes the compiler drain every load in turn).
template <typename T, int VMAX, int NT>
struct TileIo {
  static constexpr int EPS = 16 / (2 * (int)sizeof(T));  // elements per 16-byte slot
  static constexpr int SLOTS = (1 << VMAX) / EPS;
  static constexpr int ITERS = (SLOTS + NT - 1) / NT;
  uint64_t off[ITERS];
  uint32_t lslot[ITERS];
  int slots;

  template <typename G>
  __device__ inline void init(const G& g, int tid) {
    slots = (1 << g.V) / EPS;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const uint32_t j = (uint32_t)((it * NT + tid) * EPS);
      uint64_t o = 0;
      for (int b = 0; b < g.V; ++b) o |= (uint64_t)((j >> b) & 1u) << g.vpos[b];
      off[it] = o;
      lslot[it] = (j ^ swz(j, g)) / EPS;
    }
  }
  template <bool FULL>
  __device__ inline bool has(int it, int tid) const { return FULL || it * NT + tid < slots; }
};

// First tile of this workgroup in a persistent grid (each workgroup then advances by
// gridDim.x).  Workgroups are dealt round-robin over the 8 XCDs; when the grid is a multiple
// of 8, XCD x gets the contiguous range [x, x + 1) * gridDim.x / 8 of first tiles, so the tiles
// in flight on one XCD differ in their low tile-index bits.  Otherwise the concurrent tiles of
// an XCD share those bits (and the address bits they select), which on some qubit placements
// confines one XCD's traffic to a fraction of its memory channels.  Any value is a bijection
// of [0, gridDim.x), so every tile is still processed exactly once.
__device__ inline uint64_t xcd_first_tile() {
  const uint32_t gx = gridDim.x, bx = blockIdx.x;
  if (gx % 8u != 0u) return bx;
  return (uint64_t)((bx % 8u) * (gx / 8u) + bx / 8u);
}

template <typename G>
__device__ inline uint64_t tile_base(const G& g, uint64_t tile) {
  uint64_t b = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r)  // constant indices keep the run table in scalar registers
    if (r < g.nruns) b |= ((tile >> g.run_src[r]) & ((1ull << g.run_len[r]) - 1ull)) << g.run_dst[r];
  return b;
}

// Workgroup barrier for LDS traffic only: LDS writes before it are visible to every wave after
// it, while global loads and stores stay in flight across it (a full __syncthreads also waits
// for every outstanding global access, which would serialise the tile pipeline).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup barrier without memory fences, for kernels that fill LDS with direct
// global-to-LDS loads: a fence would also wait for those in-flight loads.  The empty asm
// statements keep the compiler from moving memory accesses across it; the explicit lgkmcnt(0)
// completes this wave's own LDS reads and writes first.
__device__ inline void raw_barrier() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// Wait until at most N vector-memory operations of this wave are outstanding (in issue order).
template <int N>
__device__ inline void vm_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

template <bool RAW>
__device__ inline void tile_barrier() {
  if constexpr (RAW)
    raw_barrier();
  else
    lds_barrier();
}

// Direct global-to-LDS staging (gfx950 global_load_lds_dwordx4): each lane's 16-byte load
// lands in LDS at the wave's base + 16 * lane, so LDS slot it * NT + tid is filled from the
// tile element that the swizzle maps there.  The swizzle is an involution (it only flips
// bits inside the bank window, chosen by bits above it), so the element held by LDS element j
// is j ^ X(j).  Full tiles only.
template <typename T, int VMAX, int NT>
struct TileDma {
  static constexpr int EPS = 16 / (2 * (int)sizeof(T));
  static constexpr int SLOTS = (1 << VMAX) / EPS;
  static constexpr int ITERS = SLOTS / NT;
  static_assert(SLOTS % NT == 0, "whole waves per LDS row");
  uint64_t off[ITERS];

  template <typename G>
  __device__ inline void init(const G& g, int tid) {
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const uint32_t j = (uint32_t)((it * NT + tid) * EPS);
      const uint32_t e = j ^ swz(j, g);
      uint64_t o = 0;
      for (int b = 0; b < VMAX; ++b) o |= (uint64_t)((e >> b) & 1u) << g.vpos[b];
      off[it] = o;
    }
  }
  __device__ inline void load(const T* rho, uint64_t base, u32x4* buf, int tid, int wave) const {
#pragma unroll
    for (int it = 0; it < ITERS; ++it)
      __builtin_amdgcn_global_load_lds(rho + 2 * (base + off[it]), buf + it * NT + wave * 64, 16, 0, 0);
  }
  __device__ inline void store(T* rho, uint64_t base, const u32x4* buf, int tid) const {
#pragma unroll
    for (int it = 0; it < ITERS; ++it) *reinterpret_cast<u32x4*>(rho + 2 * (base + off[it])) = buf[it * NT + tid];
  }
};

// ------------------------------------------------------------------------------------
// k = 2: real-block form.  Interleaved data is a real vector of length 32 and S the 32 x 32
// real matrix [[Sr, -Si], [Si, Sr]] (interleaved); each wave owns 16-group column blocks and
// all of S: 2 m-tiles x 8 k-steps of 16x16x4 MFMA per block.  In place, no barrier inside:
// a wave reads and writes only its own groups.  prepare() computes everything that depends
// only on the geometry and the lane (group offsets, swizzle, row offsets) once per launch.
// compute<true>: every tile holds 2^VMAX elements, so every lane of every column block is a
// group.  LDS reads are never guarded (a guarded read puts a full LDS wait before every MFMA):
// in partial tiles the lanes past the last group read group 0 and write nothing.
// ------------------------------------------------------------------------------------
template <typename T, int VMAX, int NT>
struct Op2 {
  static constexpr int kVmax = VMAX, kThreads = NT;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using c2 = typename M::c2;
  static constexpr int MT = 2, KS = 8;
  static constexpr int NW = NT / 64;
  static constexpr int NB_MAX = (1 << (VMAX - 4)) / 16;  // column blocks of a full tile
  static constexpr int NBW = (NB_MAX + NW - 1) / NW;     // column blocks per wave
  static_assert(NB_MAX % NW == 0, "full tiles give every wave the same number of blocks");
  T afr[MT][KS];
  uint32_t gj[NBW], xg[NBW];
  bool act[NBW];
  uint32_t tj1, tq;
  int nblk;

  __device__ inline void load(const T* __restrict__ frag_in, int lane) {
    const auto* frag = global_ptr(frag_in);  // device operands (kernel argument or work list)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int s = 0; s < KS; ++s) afr[m][s] = frag[(m * KS + s) * 64 + lane];
  }

  template <typename G>
  __device__ inline void prepare(const G& g, int lane, int wave) {
    const int GG = g.G;
    nblk = (GG + 15) >> 4;
    const int kk = lane >> 4;
    tj1 = (kk >> 1) ? g.tj[1] : 0u;  // tile-local part of the B row's low complex bit
    tq = g.tj[2 * kk];                // f32: outputs 2 kk and 2 kk + 1 of each m-tile
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int gi = (wave + i * NW) * 16 + (lane & 15);
      act[i] = gi < GG;
      gj[i] = act[i] ? pdep32((uint32_t)gi, g.free_mask) : 0u;
      xg[i] = swz(gj[i], g);
    }
  }

  template <bool FULL, bool RAW = false, typename G>
  __device__ inline void compute(T* ldsT, const G& g, int lane, int wave) const {
    const int cc = (lane >> 4) & 1;  // re / im of the B row
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      if (!FULL && wave + i * NW >= nblk) break;  // uniform per wave
      acc_t acc[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = acc_t{0, 0, 0, 0};
      // inactive lanes (partial tiles only) read group 0, which is in the tile, and write nothing
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint32_t e = ((g.tj[2 * s] + tj1) ^ xg[i]) + gj[i];
        const T b = ldsT[2 * e + cc];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = M::mma(afr[m][s], b, acc[m]);
      }
      if (FULL || act[i]) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          if constexpr (M::kRowsStrided) {
            // value r = real row kk + 4r of m-tile m: component cc of output a = 8m + 2r + hb
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint32_t e = ((g.tj[8 * m] + g.tj[2 * r] + tj1) ^ xg[i]) + gj[i];
              ldsT[2 * e + cc] = acc[m][r];
            }
          } else {
            // values (0,1), (2,3) = (re, im) of outputs a = 8m + 2kk and a + 1
            const uint32_t e0 = ((g.tj[8 * m] + tq) ^ xg[i]) + gj[i];
            const uint32_t e1 = ((g.tj[8 * m] + tq + g.tj[1]) ^ xg[i]) + gj[i];
            *reinterpret_cast<c2*>(ldsT + 2 * e0) = c2{acc[m][0], acc[m][1]};
            *reinterpret_cast<c2*>(ldsT + 2 * e1) = c2{acc[m][2], acc[m][3]};
          }
        }
      }
    }
  }
};

// ------------------------------------------------------------------------------------
// k = 3: 3M form, P1 = Sr xr, P2 = Si xi, P3 = (Sr + Si)(xr + xi); Re = P1 - P2,
// Im = P3 - P1 - P2: three real 64 x 64 products instead of four.  Each wave holds one
// 16-row m-tile of (Sr, Si, Sr + Si) and a share of the tile's column blocks.  compute()
// contains one LDS barrier: every wave reads the whole tile before the outputs overwrite it.
// ------------------------------------------------------------------------------------
template <typename T, int VMAX, int NT>
struct Op3 {
  static constexpr int kVmax = VMAX, kThreads = NT;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using c2 = typename M::c2;
  static constexpr int NW = NT / 64;
  static_assert(NW % 4 == 0, "four m-tiles of 16 complex rows");
  static constexpr int NPART = NW / 4;                         // waves sharing one m-tile
  static constexpr int NB_MAX = (1 << (VMAX - 6)) / 16;        // column blocks per full tile
  static constexpr int NBW = (NB_MAX + NPART - 1) / NPART;     // column blocks per wave
  static_assert(NB_MAX % NPART == 0, "full tiles give every wave the same number of blocks");
  static constexpr int KS = 16;                                // 64 complex columns, steps of 4
  T ar[KS], ai[KS], as[KS];
  uint32_t gj[NBW], xg[NBW];
  bool act[NBW];
  uint32_t tjk, trow0, tjm;
  // tile-local offsets of local-index bits 2-5 (tj[4], tj[8], tj[16], tj[32]) and of bits 0-1
  // (tj[1], tj[2]), the same in every lane: tj is linear in the local index (disjoint bits),
  // so every tj[4 s] and output-row offset is a sum of these, formed in scalar registers
  // rather than read from the geometry for every tile (in LDS, in the batched kernel)
  uint32_t tb[4], tl[2];
  int nblk;

  // tj[4 s]
  __device__ inline uint32_t tk(int s) const {
    return ((s & 1) ? tb[0] : 0u) + ((s & 2) ? tb[1] : 0u) + ((s & 4) ? tb[2] : 0u) + ((s & 8) ? tb[3] : 0u);
  }
  // tile-local offset of accumulator value r's output row within a k-step: tj[4 r] (FP64,
  // rows kk + 4 r) or tj[r] (FP32, rows 4 kk + r)
  __device__ inline uint32_t trow_of(int r) const {
    if constexpr (M::kRowsStrided) return ((r & 1) ? tb[0] : 0u) + ((r & 2) ? tb[1] : 0u);
    return ((r & 1) ? tl[0] : 0u) + ((r & 2) ? tl[1] : 0u);
  }

  __device__ inline void load(const T* __restrict__ frag_in, int lane, int wave) {
    const auto* frag = global_ptr(frag_in);  // device operands (kernel argument or work list)
    const int mt = wave & 3;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      ar[s] = frag[((mt * KS + s) * 3 + 0) * 64 + lane];
      ai[s] = frag[((mt * KS + s) * 3 + 1) * 64 + lane];
      as[s] = frag[((mt * KS + s) * 3 + 2) * 64 + lane];
    }
  }

  template <typename G>
  __device__ inline void prepare(const G& g, int lane, int wave) {
    const int GG = g.G;
    nblk = (GG + 15) >> 4;
    const int kk = lane >> 4, part = wave >> 2;
    tjk = g.tj[kk];                                      // B row 4s + kk: tj[4s] + tj[kk]
    trow0 = M::kRowsStrided ? g.tj[kk] : g.tj[4 * kk];   // output row kk + 4r (f64), 4kk + r (f32)
    tjm = g.tj[16 * (wave & 3)];                         // this wave's output m-tile
#pragma unroll
    for (int b = 0; b < 4; ++b) tb[b] = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.tj[4 << b]);
    tl[0] = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.tj[1]);
    tl[1] = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.tj[2]);
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int gi = (part + i * NPART) * 16 + (lane & 15);
      act[i] = gi < GG;
      gj[i] = act[i] ? pdep32((uint32_t)gi, g.free_mask) : 0u;
      xg[i] = swz(gj[i], g);
    }
  }

  // Out of place: reads the tile from `in`, writes the results to `out` (the same layout), so no
  // barrier is needed between the reads and the writes.
  template <bool FULL, typename G>
  __device__ inline void compute_to(const c2* in, c2* out, const G& g, int lane, int wave) const {
    const int part = wave >> 2;
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      if (!(FULL || part + i * NPART < nblk)) continue;
      acc_t p1 = acc_t{0, 0, 0, 0}, p2 = acc_t{0, 0, 0, 0}, p3 = acc_t{0, 0, 0, 0};
      // inactive lanes (partial tiles only) read group 0, which is in the tile, and write nothing
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint32_t e = ((tk(s) + tjk) ^ xg[i]) + gj[i];
        const c2 v = in[e];
        const T br = v[0], bi = v[1];
        p1 = M::mma(ar[s], br, p1);
        p2 = M::mma(ai[s], bi, p2);
        p3 = M::mma(as[s], br + bi, p3);
      }
      if (FULL || act[i]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t trow = trow0 + trow_of(r);
          const uint32_t e = ((tjm + trow) ^ xg[i]) + gj[i];
          out[e] = c2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
      }
    }
  }

  template <bool FULL, bool RAW = false, typename G>
  __device__ inline void compute(c2* ldsC, const G& g, int lane, int wave) const {
    const int part = wave >> 2;
    acc_t p1[NBW], p2[NBW], p3[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      p1[i] = acc_t{0, 0, 0, 0};
      p2[i] = acc_t{0, 0, 0, 0};
      p3[i] = acc_t{0, 0, 0, 0};
      if (FULL || part + i * NPART < nblk) {
        // inactive lanes (partial tiles only) read group 0, which is in the tile, and write nothing
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const uint32_t e = ((tk(s) + tjk) ^ xg[i]) + gj[i];
          const c2 v = ldsC[e];
          const T br = v[0], bi = v[1];
          const T bs = br + bi;
          p1[i] = M::mma(ar[s], br, p1[i]);
          p2[i] = M::mma(ai[s], bi, p2[i]);
          p3[i] = M::mma(as[s], bs, p3[i]);
        }
      }
    }
    tile_barrier<RAW>();  // every wave has read the whole tile before outputs overwrite it
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      if ((FULL || part + i * NPART < nblk) && act[i]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t trow = trow0 + trow_of(r);
          const uint32_t e = ((tjm + trow) ^ xg[i]) + gj[i];
          const T re = p1[i][r] - p2[i][r];
          const T im = p3[i][r] - p1[i][r] - p2[i][r];
          ldsC[e] = c2{re, im};
        }
      }
    }
  }
};

}  // namespace tanq
