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
// for every tile of one geometry.  FULL: the tile has all 2^VMAX elements, so no per-slot guard.
template <typename T, int VMAX, int NT, bool FULL>
struct TileIo {
  static constexpr int EPS = 16 / (2 * (int)sizeof(T));  // elements per 16-byte slot
  static constexpr int SLOTS = (1 << VMAX) / EPS;
  static constexpr int ITERS = (SLOTS + NT - 1) / NT;
  uint64_t off[ITERS];
  uint32_t lslot[ITERS];
  int slots;

  template <typename G>
  __device__ inline void init(const G& g, int tid) {
    slots = FULL ? SLOTS : (1 << g.V) / EPS;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const uint32_t j = (uint32_t)((it * NT + tid) * EPS);
      uint64_t o = 0;
      for (int b = 0; b < (FULL ? VMAX : g.V); ++b) o |= (uint64_t)((j >> b) & 1u) << g.vpos[b];
      off[it] = o;
      lslot[it] = (j ^ swz(j, g)) / EPS;
    }
  }
  __device__ inline bool has(int it, int tid) const { return FULL || it * NT + tid < slots; }
};

template <typename G>
__device__ inline uint64_t tile_base(const G& g, uint64_t tile) {
  uint64_t b = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r)  // constant indices keep the run table in scalar registers
    if (r < g.nruns) b |= ((tile >> g.run_src[r]) & ((1ull << g.run_len[r]) - 1ull)) << g.run_dst[r];
  return b;
}

// ------------------------------------------------------------------------------------
// k = 2: real-block form.  Interleaved data is a real vector of length 32 and S the 32 x 32
// real matrix [[Sr, -Si], [Si, Sr]] (interleaved); each wave owns 16-group column blocks and
// all of S: 2 m-tiles x 8 k-steps of 16x16x4 MFMA per block.  In place, no barrier inside:
// a wave reads and writes only its own groups.
// ------------------------------------------------------------------------------------
template <typename T, int NT>
struct Op2 {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using c2 = typename M::c2;
  static constexpr int MT = 2, KS = 8;
  T afr[MT][KS];

  __device__ inline void load(const T* __restrict__ frag, int lane) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int s = 0; s < KS; ++s) afr[m][s] = frag[(m * KS + s) * 64 + lane];
  }

  template <typename G>
  __device__ inline void compute(T* ldsT, const G& g, int lane, int wave) const {
    constexpr int NW = NT / 64;
    const int GG = g.G;
    const int nblk = (GG + 15) >> 4;
    const int kk = lane >> 4;
    const int hb = kk >> 1;                  // low bit of the B row's complex index
    const int cc = kk & 1;                   // re / im of the B row
    const uint32_t tj1 = hb ? g.tj[1] : 0u;  // tile-local part contributed by that bit
    const uint32_t tq = g.tj[2 * kk];        // f32: outputs 2 kk and 2 kk + 1 of each m-tile
    for (int nb = wave; nb < nblk; nb += NW) {
      const int gi = nb * 16 + (lane & 15);
      const bool act = gi < GG;
      const uint32_t gj = act ? pdep32((uint32_t)gi, g.free_mask) : 0u;
      const uint32_t xg = swz(gj, g);
      acc_t acc[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint32_t e = ((g.tj[2 * s] + tj1) ^ xg) + gj;
        const T b = act ? ldsT[2 * e + cc] : T(0);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = M::mma(afr[m][s], b, acc[m]);
      }
      if (act) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          if constexpr (M::kRowsStrided) {
            // value r = real row kk + 4r of m-tile m: component cc of output a = 8m + 2r + hb
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint32_t e = ((g.tj[8 * m] + g.tj[2 * r] + tj1) ^ xg) + gj;
              ldsT[2 * e + cc] = acc[m][r];
            }
          } else {
            // values (0,1), (2,3) = (re, im) of outputs a = 8m + 2kk and a + 1
            const uint32_t e0 = ((g.tj[8 * m] + tq) ^ xg) + gj;
            const uint32_t e1 = ((g.tj[8 * m] + tq + g.tj[1]) ^ xg) + gj;
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
// contains one barrier: every wave reads the whole tile before the outputs overwrite it.
// ------------------------------------------------------------------------------------
template <typename T, int VMAX, int NT>
struct Op3 {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using c2 = typename M::c2;
  static constexpr int NW = NT / 64;
  static_assert(NW % 4 == 0, "four m-tiles of 16 complex rows");
  static constexpr int NPART = NW / 4;                         // waves sharing one m-tile
  static constexpr int NB_MAX = (1 << (VMAX - 6)) / 16;        // column blocks per full tile
  static constexpr int NBW = (NB_MAX + NPART - 1) / NPART;     // column blocks per wave
  static constexpr int KS = 16;                                // 64 complex columns, steps of 4
  T ar[KS], ai[KS], as[KS];

  __device__ inline void load(const T* __restrict__ frag, int lane, int wave) {
    const int mt = wave & 3;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      ar[s] = frag[((mt * KS + s) * 3 + 0) * 64 + lane];
      ai[s] = frag[((mt * KS + s) * 3 + 1) * 64 + lane];
      as[s] = frag[((mt * KS + s) * 3 + 2) * 64 + lane];
    }
  }

  template <typename G>
  __device__ inline void compute(c2* ldsC, const G& g, int lane, int wave) const {
    const int mt = wave & 3, part = wave >> 2;
    const int GG = g.G;
    const int nblk = (GG + 15) >> 4;
    const int kk = lane >> 4;
    const uint32_t tjk = g.tj[kk];       // B row 4s + kk: tj[4s] + tj[kk]
    const uint32_t tj4k = g.tj[4 * kk];  // f32 output rows 4 kk + r
    const uint32_t tjm = g.tj[16 * mt];  // this wave's output block
    acc_t p1[NBW], p2[NBW], p3[NBW];
    uint32_t gjs[NBW], xgs[NBW];
    bool acts[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int nb = part + i * NPART;
      const int gi = nb * 16 + (lane & 15);
      acts[i] = nb < nblk && gi < GG;
      gjs[i] = acts[i] ? pdep32((uint32_t)gi, g.free_mask) : 0u;
      xgs[i] = swz(gjs[i], g);
      p1[i] = acc_t{0, 0, 0, 0};
      p2[i] = acc_t{0, 0, 0, 0};
      p3[i] = acc_t{0, 0, 0, 0};
      if (nb < nblk) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const uint32_t e = ((g.tj[4 * s] + tjk) ^ xgs[i]) + gjs[i];
          const c2 v = acts[i] ? ldsC[e] : c2{0, 0};
          const T br = v[0], bi = v[1];
          const T bs = br + bi;
          p1[i] = M::mma(ar[s], br, p1[i]);
          p2[i] = M::mma(ai[s], bi, p2[i]);
          p3[i] = M::mma(as[s], bs, p3[i]);
        }
      }
    }
    __syncthreads();  // every wave has read the whole tile before outputs overwrite it
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      if (acts[i]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // output row within the m-tile: kk + 4r (f64) or 4kk + r (f32)
          const uint32_t trow = M::kRowsStrided ? (tjk + g.tj[4 * r]) : (tj4k + g.tj[r]);
          const uint32_t e = ((tjm + trow) ^ xgs[i]) + gjs[i];
          const T re = p1[i][r] - p2[i][r];
          const T im = p3[i][r] - p1[i][r] - p2[i][r];
          ldsC[e] = c2{re, im};
        }
      }
    }
  }
};

}  // namespace tanq
