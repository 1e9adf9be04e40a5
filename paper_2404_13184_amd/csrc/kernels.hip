// HIP kernels of libtanq for gfx950 (CDNA4, wave64).
//
// Hot path: applying a k-qubit superoperator S (4^k x 4^k complex) to vec(rho) in place,
// i.e. the batched GEMM [4^k x 4^k] x [4^k x 4^(n-k)] whose columns are the groups of
// amplitudes differing only in the 2k target bits (Sec. 3.1 "im2col" view; Sec. 3.2 maps
// the 2-qubit case onto FP64 tensor cores).
//
// gfx950 design:
//   * A workgroup owns a tile of 2^V elements: all 2k target bits plus the lowest free bits,
//     so every group lies inside one tile and the tile is a union of long contiguous runs of
//     memory.  Tiles are read and written with 16-byte per-lane accesses (fully coalesced),
//     staged through LDS, and the grid is persistent (grid-stride over tiles).
//   * The complex GEMM is done on MFMA in real-block form: with interleaved (re, im) data,
//     x (4^k complex) is a 2*4^k real vector and S acts as the real matrix
//     [[Sr, -Si], [Si, Sr]] interleaved, so the B operand is read straight from the
//     interleaved tile.  FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32, both
//     accumulating in their own precision.
//   * The A operand (the superoperator) is pre-packed in the MFMA lane layout by the pack
//     kernel and held in VGPRs for the whole launch.
//   * k = 2: each wave owns whole groups (16 per MFMA column block) and holds all of S.
//     k = 3: S is 128 x 128 real, too large for one wave's registers, so each of 8 waves
//     holds a 16-row slice of S and reads every group of the tile.
//   * k = 1 (the paper's C1 gate, which it keeps off the tensor cores) is a VALU kernel
//     over the paper's strided index map s_i.
#include <cstring>

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
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  using c2 = f32x2;
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

// ------------------------------------------------------------------------------------
// MFMA apply kernel, k = 2 and k = 3
// ------------------------------------------------------------------------------------

// Store one m-tile of accumulators (real-block rows 16 mt .. 16 mt + 15, i.e. complex
// outputs a = a0 .. a0 + 7 with a0 = 8 mt) of this lane's group into the LDS tile.
//   f64: value r is row (l/16) + 4r: component cc = (l/16) & 1 of complex output
//        a0 + 2r + hb; its tile-local index is tj[a0] + tj[2r] + lp (lp = group + tj(hb)).
//   f32: values (0,1) and (2,3) are the (re, im) pairs of outputs a0 + 2(l/16) and that + 1;
//        tile-local index tj[a0] + tq (tq = tj[2(l/16)] + group) and that + tj[1].
template <typename T, typename Acc>
__device__ inline void write_outputs(T* ldsT, const Acc& acc, const uint32_t* tj, int a0, uint32_t lp, uint32_t tqg,
                                     int cc) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int r = 0; r < 4; ++r) ldsT[2 * (tj[a0] + tj[2 * r] + lp) + cc] = acc[r];
  } else {
    using c2 = typename Mfma<T>::c2;
    const uint32_t e0 = tj[a0] + tqg;
    const uint32_t e1 = e0 + tj[1];
    *reinterpret_cast<c2*>(ldsT + 2 * e0) = c2{acc[0], acc[1]};
    *reinterpret_cast<c2*>(ldsT + 2 * e1) = c2{acc[2], acc[3]};
  }
}

// FULL: the tile has all 2^VMAX elements (every register size but the smallest), so the
// load/store phases are straight-line code with no per-slot guards; that lets the compiler
// wait only for the prefetched loads at the top of the loop and leave the previous tile's
// stores in flight.
template <typename T, int K, int VMAX, int NT, bool FULL>
__global__ __launch_bounds__(NT) void apply_mfma_kernel(T* __restrict__ rho, const T* __restrict__ frag,
                                                        const ApplyGeom g) {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int NW = NT / 64;
  constexpr int D = 1 << (2 * K);  // superoperator dimension (complex)
  constexpr int R2 = 2 * D;        // real-block dimension
  constexpr int MT = R2 / 16;      // 16-row m-tiles
  constexpr int KS = R2 / 4;       // 4-deep k-steps
  constexpr int MTW = (K == 2) ? MT : MT / NW;  // m-tiles held by one wave
  static_assert(K == 2 || MT % NW == 0, "k = 3 splits the m-tiles evenly over the waves");
  constexpr int EPS = 16 / (2 * (int)sizeof(T));  // elements per 16-byte slot
  constexpr int SLOTS = (1 << VMAX) / EPS;
  constexpr int ITERS = (SLOTS + NT - 1) / NT;
  constexpr int NBMAX = (K == 3) ? (((1 << (VMAX - 2 * K)) + 15) / 16) : 1;

  __shared__ u32x4 lds[SLOTS];
  T* ldsT = reinterpret_cast<T*>(lds);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int slots = FULL ? SLOTS : (1 << g.V) / EPS;

  // element offset of each 16-byte slot this thread moves (identical for every tile)
  uint64_t off[ITERS];
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const uint32_t j = (uint32_t)((it * NT + tid) * EPS);
    uint64_t o = 0;
    for (int b = 0; b < (FULL ? VMAX : g.V); ++b) o |= (uint64_t)((j >> b) & 1u) << g.vpos[b];
    off[it] = o;
  }

  // A operand: this wave's slice of the packed superoperator
  const int mt0 = (K == 2) ? 0 : wave * MTW;
  T afr[MTW][KS];
#pragma unroll
  for (int m = 0; m < MTW; ++m)
#pragma unroll
    for (int s = 0; s < KS; ++s) afr[m][s] = frag[((mt0 + m) * KS + s) * 64 + lane];

  const int G = g.G;
  const int nblk = (G + 15) >> 4;
  const int hb = (lane >> 5) & 1;          // low bit of the B row's complex index
  const int cc = (lane >> 4) & 1;          // re / im of the B row
  const uint32_t tj1 = hb ? g.tj[1] : 0u;  // tile-local part contributed by that bit
  const uint32_t tq = g.tj[2 * (lane >> 4)];  // f32 output rows 4*(lane>>4) .. +3

  // constant indices keep the run table in scalar registers (loaded once)
  auto tile_base = [&](uint64_t tile) {
    uint64_t b = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r < g.nruns) b |= ((tile >> g.run_src[r]) & ((1ull << g.run_len[r]) - 1ull)) << g.run_dst[r];
    return b;
  };

  // Software pipeline: the next tile's global loads are in flight while this tile is
  // multiplied and written back.  The loop is rotated so that the wait for those loads
  // comes after this tile's stores have been issued: the vector-memory counter then only
  // has to drain to the number of stores, and the stores overlap the next tile's work.
  uint64_t tile = blockIdx.x;
  if (tile >= g.ntiles) return;  // uniform per workgroup
  uint64_t cur = tile_base(tile);
  u32x4 buf[ITERS];
#pragma unroll
  for (int it = 0; it < ITERS; ++it)
    if (FULL || it * NT + tid < slots) buf[it] = *reinterpret_cast<const u32x4*>(rho + 2 * (cur + off[it]));
#pragma unroll
  for (int it = 0; it < ITERS; ++it)
    if (FULL || it * NT + tid < slots) lds[it * NT + tid] = buf[it];
  __syncthreads();

  for (;;) {
    const uint64_t next = tile + gridDim.x;
    const bool more = next < g.ntiles;
    uint64_t nbase = 0;
    if (more) {
      nbase = tile_base(next);
#pragma unroll
      for (int it = 0; it < ITERS; ++it)
        if (FULL || it * NT + tid < slots) buf[it] = *reinterpret_cast<const u32x4*>(rho + 2 * (nbase + off[it]));
    }

    if constexpr (K == 2) {
      for (int nb = wave; nb < nblk; nb += NW) {
        const int gi = nb * 16 + (lane & 15);
        const bool act = gi < G;
        const uint32_t gj = act ? pdep32((uint32_t)gi, g.free_mask) : 0u;
        const uint32_t lp = gj | tj1;
        acc_t acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const T b = act ? ldsT[2 * (g.tj[2 * s] + lp) + cc] : T(0);
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m] = M::mma(afr[m][s], b, acc[m]);
        }
        if (act) {
#pragma unroll
          for (int m = 0; m < MT; ++m) write_outputs<T>(ldsT, acc[m], g.tj, 8 * m, lp, tq + gj, cc);
        }
      }
    } else {
      acc_t acc[NBMAX][MTW];
      uint32_t gjs[NBMAX];
#pragma unroll
      for (int nb = 0; nb < NBMAX; ++nb) {
        const int gi = nb * 16 + (lane & 15);
        gjs[nb] = (nb < nblk && gi < G) ? pdep32((uint32_t)gi, g.free_mask) : 0xffffffffu;
#pragma unroll
        for (int m = 0; m < MTW; ++m) acc[nb][m] = acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int nb = 0; nb < NBMAX; ++nb) {
        if (nb < nblk) {
          const bool act = gjs[nb] != 0xffffffffu;
          const uint32_t lp = (act ? gjs[nb] : 0u) + tj1;
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const T b = act ? ldsT[2 * (g.tj[2 * s] + lp) + cc] : T(0);
#pragma unroll
            for (int m = 0; m < MTW; ++m) acc[nb][m] = M::mma(afr[m][s], b, acc[nb][m]);
          }
        }
      }
      __syncthreads();  // every wave has read the whole tile before outputs overwrite it
#pragma unroll
      for (int nb = 0; nb < NBMAX; ++nb) {
        if (nb < nblk && gjs[nb] != 0xffffffffu) {
#pragma unroll
          for (int m = 0; m < MTW; ++m)
            write_outputs<T>(ldsT, acc[nb][m], g.tj, 8 * (mt0 + m), gjs[nb] + tj1, tq + gjs[nb], cc);
        }
      }
    }
    __syncthreads();

#pragma unroll
    for (int it = 0; it < ITERS; ++it)
      if (FULL || it * NT + tid < slots) *reinterpret_cast<u32x4*>(rho + 2 * (cur + off[it])) = lds[it * NT + tid];
    if (!more) break;
    __syncthreads();  // every store-phase LDS read is done before the next tile lands
#pragma unroll
    for (int it = 0; it < ITERS; ++it)
      if (FULL || it * NT + tid < slots) lds[it * NT + tid] = buf[it];
    __syncthreads();
    tile = next;
    cur = nbase;
  }
}

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
// initialisation
// ------------------------------------------------------------------------------------

template <typename T>
__global__ void init_zero_kernel(T* __restrict__ rho, uint64_t nreal) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nreal; i += (uint64_t)gridDim.x * blockDim.x)
    rho[i] = (i == 0) ? T(1) : T(0);
}

__device__ inline uint64_t splitmix64(uint64_t c) {
  uint64_t z = c + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void fill_random_kernel(T* __restrict__ rho, uint64_t nel, uint64_t seed) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = (seed << 40) + e;
    const double re = (double)(splitmix64(2 * x) >> 11) * 0x1.0p-53 - 0.5;
    const double im = (double)(splitmix64(2 * x + 1) >> 11) * 0x1.0p-53 - 0.5;
    rho[2 * e] = (T)re;
    rho[2 * e + 1] = (T)im;
  }
}

template <typename T>
__global__ void gather_kernel(const T* __restrict__ rho, const uint64_t* __restrict__ idx, uint64_t count,
                              T* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = idx[i];
    out[2 * i] = rho[2 * e];
    out[2 * i + 1] = rho[2 * e + 1];
  }
}

// ------------------------------------------------------------------------------------
// superoperator construction, composition and packing (FP64)
// ------------------------------------------------------------------------------------

// S[(ar + 2^j ac), (br + 2^j bc)] = sum_i conj(K_i[ac][bc]) K_i[ar][br]   (Sec. 3.1)
__global__ void build_superops_kernel(const FuseOpDev* __restrict__ ops, const double* __restrict__ kraus,
                                      double* __restrict__ sops) {
  const FuseOpDev op = ops[blockIdx.x];
  const int j = op.j, d = 1 << j, dd = d * d;
  const double* K = kraus + 2 * op.kraus_off;
  double* S = sops + 2 * op.sop_off;
  for (int e = threadIdx.x; e < dd * dd; e += blockDim.x) {
    const int a = e / dd, b = e % dd;
    const int ar = a & (d - 1), ac = a >> j, br = b & (d - 1), bc = b >> j;
    double sr = 0.0, si = 0.0;
    for (int i = 0; i < op.m; ++i) {
      const double* Ki = K + 2 * (size_t)i * d * d;
      const double xr = Ki[2 * (ac * d + bc)], xi = -Ki[2 * (ac * d + bc) + 1];  // conj
      const double yr = Ki[2 * (ar * d + br)], yi = Ki[2 * (ar * d + br) + 1];
      sr += xr * yr - xi * yi;
      si += xr * yi + xi * yr;
    }
    S[2 * e] = sr;
    S[2 * e + 1] = si;
  }
}

// One workgroup per block: M <- S_op(embedded) M for each operation, starting from M = I.
// Column c of the result is vec of the block's action on the basis operator with vec
// index c, so the final M is S_blk = S_last ... S_first.
template <int KMAX>
__global__ __launch_bounds__(256) void compose_kernel(const FuseBlockDev* __restrict__ blocks,
                                                      const FuseOpDev* __restrict__ ops,
                                                      const double* __restrict__ sops, double* __restrict__ out) {
  constexpr int DMAX = 1 << (2 * KMAX);
  __shared__ f64x2 buf[2][DMAX * DMAX];
  __shared__ uint32_t dep[64];
  const FuseBlockDev blk = blocks[blockIdx.x];
  const int k = blk.k, Dk = 1 << (2 * k);
  f64x2* Min = buf[0];
  f64x2* Mout = buf[1];
  for (int e = threadIdx.x; e < Dk * Dk; e += blockDim.x) Min[e] = f64x2{(e / Dk) == (e % Dk) ? 1.0 : 0.0, 0.0};
  __syncthreads();
  for (int oi = 0; oi < blk.op_count; ++oi) {
    const FuseOpDev op = ops[blk.op_begin + oi];
    const int j = op.j, Dj = 1 << (2 * j);
    uint32_t tmask = 0;
    for (int t = 0; t < j; ++t) tmask |= (1u << op.pos[t]) | (1u << (k + op.pos[t]));
    for (int b = threadIdx.x; b < Dj; b += blockDim.x) {
      uint32_t r = 0;
      for (int t = 0; t < j; ++t) {
        if ((b >> t) & 1) r |= 1u << op.pos[t];
        if ((b >> (j + t)) & 1) r |= 1u << (k + op.pos[t]);
      }
      dep[b] = r;
    }
    __syncthreads();
    const double* S = sops + 2 * op.sop_off;
    for (int e = threadIdx.x; e < Dk * Dk; e += blockDim.x) {
      const int a = e / Dk, c = e % Dk;
      uint32_t aloc = 0;
      for (int t = 0; t < j; ++t) {
        aloc |= (uint32_t)((a >> op.pos[t]) & 1) << t;
        aloc |= (uint32_t)((a >> (k + op.pos[t])) & 1) << (j + t);
      }
      const uint32_t abase = (uint32_t)a & ~tmask;
      double sr = 0.0, si = 0.0;
      for (int b = 0; b < Dj; ++b) {
        const double xr = S[2 * (aloc * Dj + b)], xi = S[2 * (aloc * Dj + b) + 1];
        const f64x2 y = Min[(abase | dep[b]) * Dk + c];
        sr += xr * y[0] - xi * y[1];
        si += xr * y[1] + xi * y[0];
      }
      Mout[e] = f64x2{sr, si};
    }
    __syncthreads();
    f64x2* t = Min;
    Min = Mout;
    Mout = t;
  }
  double* O = out + 2 * blk.out_off;
  for (int e = threadIdx.x; e < Dk * Dk; e += blockDim.x) {
    O[2 * e] = Min[e][0];
    O[2 * e + 1] = Min[e][1];
  }
}

// Real-block fragments: R[m'][k'] for m' = 2a + cm, k' = 2b + ck is
//   (cm, ck) = (0,0): Re S[a][b]   (0,1): -Im S[a][b]   (1,0): Im S[a][b]   (1,1): Re S[a][b]
// stored as frag[(mt * KS + ks) * 64 + lane] = R[16 mt + lane % 16][4 ks + lane / 16].
template <typename T>
__device__ void pack_block(int k, const double* __restrict__ S, T* __restrict__ P) {
  const int D = 1 << (2 * k);
  const int R2 = 2 * D, KS = R2 / 4, MT = R2 / 16;
  for (int e = threadIdx.x; e < MT * KS * 64; e += blockDim.x) {
    const int lane = e & 63, rest = e >> 6;
    const int ks = rest % KS, mt = rest / KS;
    const int mrow = 16 * mt + (lane & 15), kcol = 4 * ks + (lane >> 4);
    const int a = mrow >> 1, cm = mrow & 1, b = kcol >> 1, ck = kcol & 1;
    const double re = S[2 * (a * D + b)], im = S[2 * (a * D + b) + 1];
    const double v = (cm == ck) ? re : (cm == 0 ? -im : im);
    P[e] = (T)v;
  }
}

template <typename T>
__global__ void pack_kernel(const FuseBlockDev* __restrict__ blocks, const double* __restrict__ raw,
                            unsigned char* __restrict__ packed) {
  const FuseBlockDev blk = blocks[blockIdx.x];
  const double* S = raw + 2 * blk.out_off;
  if (blk.k == 1) {
    double* P = reinterpret_cast<double*>(packed + blk.pack_off);
    for (int e = threadIdx.x; e < 32; e += blockDim.x) P[e] = S[e];
  } else {
    pack_block<T>(blk.k, S, reinterpret_cast<T*>(packed + blk.pack_off));
  }
}

template <typename T>
__global__ void pack_one_kernel(int k, const double* __restrict__ raw, unsigned char* __restrict__ packed) {
  if (k == 1) {
    double* P = reinterpret_cast<double*>(packed);
    for (int e = threadIdx.x; e < 32; e += blockDim.x) P[e] = raw[e];
  } else {
    pack_block<T>(k, raw, reinterpret_cast<T*>(packed));
  }
}

// ------------------------------------------------------------------------------------
// FP64 reductions
// ------------------------------------------------------------------------------------

constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

// p[x] = Re rho[x][x] = Re vec[x (2^n + 1)]; partial trace per workgroup
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void diag_kernel(const T* __restrict__ rho, int n, double* __restrict__ p,
                                                          double* __restrict__ partials) {
  __shared__ double sh[RED_THREADS / 64];
  const uint64_t dim = 1ull << n;
  double acc = 0.0;
  for (uint64_t x = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * RED_THREADS) {
    const double v = (double)rho[2 * (x * (dim + 1))];
    p[x] = v;
    acc += v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void sum_partials_kernel(const double* __restrict__ partials, int count, int nstr, double* __restrict__ out) {
  // one thread per output value; fixed summation order
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nstr) {
    double t = 0.0;
    for (int b = 0; b < count; ++b) t += partials[(size_t)i * count + b];
    out[i] = t;
  }
}

__global__ void renormalize_kernel(double* __restrict__ p, uint64_t dim, const double* __restrict__ tr) {
  const double inv = 1.0 / tr[0];
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * blockDim.x)
    p[x] *= inv;
}

// Tr(P rho) = sum_s phase(s) rho[s][s ^ xmask],  phase(s) = i^{#Y} (-1)^{popcount(s & zmask)}
// masks[3 i + 0] = xmask (X or Y), masks[3 i + 1] = zmask (Z or Y), masks[3 i + 2] = #Y mod 4
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void pauli_kernel(const T* __restrict__ rho, int n,
                                                           const uint64_t* __restrict__ masks,
                                                           double* __restrict__ partials) {
  __shared__ double sh[RED_THREADS / 64];
  const int si = blockIdx.y;
  const uint64_t xm = masks[3 * si], zm = masks[3 * si + 1];
  const int ny = (int)masks[3 * si + 2];
  const uint64_t dim = 1ull << n;
  double ar = 0.0, ai = 0.0;
  for (uint64_t s = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; s < dim; s += (uint64_t)gridDim.x * RED_THREADS) {
    const uint64_t e = s + ((s ^ xm) << n);
    const double vr = (double)rho[2 * e], vi = (double)rho[2 * e + 1];
    const double sg = (__popcll(s & zm) & 1) ? -1.0 : 1.0;
    ar += sg * vr;
    ai += sg * vi;
  }
  // multiply by i^{#Y}
  double pr = ar, pi = ai;
  if (ny == 1) { pr = -ai; pi = ar; }
  else if (ny == 2) { pr = -ar; pi = -ai; }
  else if (ny == 3) { pr = ai; pi = -ar; }
  const double tr = block_sum(pr, sh);
  const double ti = block_sum(pi, sh);
  if (threadIdx.x == 0) {
    partials[((size_t)si * 2 + 0) * gridDim.x + blockIdx.x] = tr;
    partials[((size_t)si * 2 + 1) * gridDim.x + blockIdx.x] = ti;
  }
}

// ------------------------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------------------------

int device_cu_count() {
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

ApplyGeom make_apply_geom(int n, int k, const int* q, int vbits) {
  ApplyGeom g;
  std::memset(&g, 0, sizeof(g));
  const int nb = 2 * n;
  int V = vbits < nb ? vbits : nb;
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
  // tile-local positions of the target bits and the group (free) mask
  int tpos[6];
  uint32_t tmask_local = 0;
  for (int t = 0; t < 2 * k; ++t)
    for (int b = 0; b < V; ++b)
      if (g.vpos[b] == tgt[t]) {
        tpos[t] = b;
        tmask_local |= 1u << b;
      }
  g.free_mask = ((V >= 32) ? 0xffffffffu : ((1u << V) - 1u)) & ~tmask_local;
  const int D = 1 << (2 * k);
  for (int l = 0; l < D; ++l) {
    uint32_t r = 0;
    for (int t = 0; t < 2 * k; ++t)
      if ((l >> t) & 1) r |= 1u << tpos[t];
    g.tj[l] = r;
  }
  g.G = 1 << (V - 2 * k);
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
static int persistent_grid(KernelT kernel, int threads, uint64_t ntiles) {
  int per_cu = 0;
  TANQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
  if (per_cu < 1) per_cu = 1;
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)per_cu;
  return (int)(ntiles < cap ? ntiles : cap);
}

template <typename T, int K, int VMAX, int NT, bool FULL>
static void launch_mfma_shape(const ApplyGeom& g, void* rho, const void* frag, hipStream_t s) {
  auto kern = apply_mfma_kernel<T, K, VMAX, NT, FULL>;
  static thread_local int grid_cap_dev = -1;
  static thread_local uint64_t grid_cap = 0;
  int dev = 0;
  TANQ_HIP(hipGetDevice(&dev));
  if (grid_cap_dev != dev) {
    grid_cap = (uint64_t)persistent_grid(kern, NT, ~0ull >> 1);
    grid_cap_dev = dev;
  }
  const uint64_t grid = g.ntiles < grid_cap ? g.ntiles : grid_cap;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, (T*)rho, (const T*)frag, g);
  TANQ_HIP(hipGetLastError());
}

template <typename T, int K, int VMAX, int NT>
static void launch_mfma(void* rho, int n, const int* qubits, const void* frag, hipStream_t s) {
  const ApplyGeom g = make_apply_geom(n, K, qubits, VMAX);
  if (g.V == VMAX)
    launch_mfma_shape<T, K, VMAX, NT, true>(g, rho, frag, s);
  else
    launch_mfma_shape<T, K, VMAX, NT, false>(g, rho, frag, s);
}

typedef void (*apply_fn)(void*, int, const int*, const void*, hipStream_t);

struct VariantEntry {
  int k;
  tanq_prec p;
  int tile_bits;
  int threads;
  apply_fn fn;
};

// Apply-kernel variants (tile shape x workgroup size); the first of each (k, precision) is
// the default until the autotuner or the caller selects another.
static const VariantEntry kVariants[] = {
    {2, TANQ_F64, 10, 256, launch_mfma<double, 2, 10, 256>},
    {2, TANQ_F64, 11, 256, launch_mfma<double, 2, 11, 256>},
    {2, TANQ_F64, 11, 512, launch_mfma<double, 2, 11, 512>},
    {2, TANQ_F64, 12, 512, launch_mfma<double, 2, 12, 512>},
    {2, TANQ_F32, 11, 256, launch_mfma<float, 2, 11, 256>},
    {2, TANQ_F32, 12, 256, launch_mfma<float, 2, 12, 256>},
    {2, TANQ_F32, 12, 512, launch_mfma<float, 2, 12, 512>},
    {2, TANQ_F32, 13, 512, launch_mfma<float, 2, 13, 512>},
    {3, TANQ_F64, 12, 512, launch_mfma<double, 3, 12, 512>},
    {3, TANQ_F64, 12, 256, launch_mfma<double, 3, 12, 256>},
    {3, TANQ_F32, 12, 512, launch_mfma<float, 3, 12, 512>},
    {3, TANQ_F32, 13, 512, launch_mfma<float, 3, 13, 512>},
    {3, TANQ_F32, 12, 256, launch_mfma<float, 3, 12, 256>},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

// selected variant per (k, precision), as an index among that pair's variants
static int g_selected[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};

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

bool variant_describe(int k, tanq_prec p, int local, int* tile_bits, int* threads) {
  const int gi = variant_global_index(k, p, local);
  if (gi < 0) return false;
  if (tile_bits) *tile_bits = kVariants[gi].tile_bits;
  if (threads) *threads = kVariants[gi].threads;
  return true;
}

bool variant_select(int k, tanq_prec p, int local) {
  if (variant_global_index(k, p, local) < 0) return false;
  g_selected[k][p == TANQ_F64 ? 0 : 1] = local;
  return true;
}

int variant_selected(int k, tanq_prec p) { return g_selected[k][p == TANQ_F64 ? 0 : 1]; }

void launch_apply(void* rho, int n, tanq_prec p, int k, const int* qubits, const void* packed, hipStream_t s) {
  if (k == 1) {
    C1Geom g{1ull << (2 * (n - 1)), qubits[0], n};
    uint64_t blocks = (g.ngroups + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 32;
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
  const int gi = variant_global_index(k, p, variant_selected(k, p));
  kVariants[gi].fn(rho, n, qubits, packed, s);
}

void launch_init_zero(void* rho, int n, tanq_prec p, hipStream_t s) {
  const uint64_t nreal = 2ull << (2 * n);
  uint64_t blocks = (nreal + 255) / 256;
  const uint64_t cap = (uint64_t)device_cu_count() * 64;
  if (blocks > cap) blocks = cap;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(init_zero_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)rho, nreal);
  else
    hipLaunchKernelGGL(init_zero_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)rho, nreal);
  TANQ_HIP(hipGetLastError());
}

void launch_fill_random(void* rho, int n, tanq_prec p, uint64_t seed, hipStream_t s) {
  const uint64_t nel = 1ull << (2 * n);
  uint64_t blocks = (nel + 255) / 256;
  const uint64_t cap = (uint64_t)device_cu_count() * 64;
  if (blocks > cap) blocks = cap;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(fill_random_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)rho, nel, seed);
  else
    hipLaunchKernelGGL(fill_random_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)rho, nel, seed);
  TANQ_HIP(hipGetLastError());
}

void launch_gather(const void* rho, tanq_prec p, const uint64_t* idx_dev, size_t count, void* out_dev,
                   hipStream_t s) {
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)rho, idx_dev,
                       (uint64_t)count, (double*)out_dev);
  else
    hipLaunchKernelGGL(gather_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)rho, idx_dev,
                       (uint64_t)count, (float*)out_dev);
  TANQ_HIP(hipGetLastError());
}

void launch_build_superops(const FuseOpDev* ops, int nops, const double* kraus, double* sops, hipStream_t s) {
  if (nops <= 0) return;
  hipLaunchKernelGGL(build_superops_kernel, dim3(nops), dim3(256), 0, s, ops, kraus, sops);
  TANQ_HIP(hipGetLastError());
}

void launch_compose(const FuseBlockDev* blocks, int nblocks, int max_k, const FuseOpDev* ops, const double* sops,
                    double* out, hipStream_t s) {
  if (nblocks <= 0) return;
  if (max_k <= 2)
    hipLaunchKernelGGL(compose_kernel<2>, dim3(nblocks), dim3(256), 0, s, blocks, ops, sops, out);
  else
    hipLaunchKernelGGL(compose_kernel<3>, dim3(nblocks), dim3(256), 0, s, blocks, ops, sops, out);
  TANQ_HIP(hipGetLastError());
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

int reduce_partials() { return RED_BLOCKS * 2 * 64; }

static int red_blocks(uint64_t dim) {
  uint64_t b = (dim + RED_THREADS - 1) / RED_THREADS;
  return (int)(b < (uint64_t)RED_BLOCKS ? b : (uint64_t)RED_BLOCKS);
}

void launch_diag(const void* rho, int n, tanq_prec p, double* probs_dev, double* partials, double* result_dev,
                 int renormalize, hipStream_t s) {
  const uint64_t dim = 1ull << n;
  const int nb = red_blocks(dim);
  if (p == TANQ_F64)
    hipLaunchKernelGGL(diag_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, s, (const double*)rho, n, probs_dev,
                       partials);
  else
    hipLaunchKernelGGL(diag_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, s, (const float*)rho, n, probs_dev,
                       partials);
  TANQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partials, nb, 1, result_dev);
  TANQ_HIP(hipGetLastError());
  if (renormalize) {
    hipLaunchKernelGGL(renormalize_kernel, dim3(nb), dim3(RED_THREADS), 0, s, probs_dev, dim, result_dev);
    TANQ_HIP(hipGetLastError());
  }
}

void launch_pauli(const void* rho, int n, tanq_prec p, int count, const uint64_t* masks_dev, double* partials,
                  double* result_dev, hipStream_t s) {
  const uint64_t dim = 1ull << n;
  int nb = red_blocks(dim);
  // partials holds 2 * count * nb doubles
  const int maxnb = reduce_partials() / (2 * count);
  if (nb > maxnb) nb = maxnb < 1 ? 1 : maxnb;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(pauli_kernel<double>, dim3(nb, count), dim3(RED_THREADS), 0, s, (const double*)rho, n,
                       masks_dev, partials);
  else
    hipLaunchKernelGGL(pauli_kernel<float>, dim3(nb, count), dim3(RED_THREADS), 0, s, (const float*)rho, n,
                       masks_dev, partials);
  TANQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3((2 * count + 63) / 64), dim3(64), 0, s, partials, nb, 2 * count,
                     result_dev);
  TANQ_HIP(hipGetLastError());
}

}  // namespace tanq
