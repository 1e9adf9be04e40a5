// Auxiliary HIP kernels of libtanq (gfx950): state initialisation and sampling, superoperator
// construction and FP64 composition for fusion, and FP64 reductions.  The apply kernels (the
// hot path) and the packing of superoperators into their operand layouts are in apply.hip.
#include <cstring>

#include "internal.hpp"

namespace tanq {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// initialisation
// ------------------------------------------------------------------------------------

template <typename T>
__global__ void init_zero_kernel(T* __restrict__ rho, uint64_t nreal) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nreal; i += (uint64_t)gridDim.x * blockDim.x)
    rho[i] = (i == 0) ? T(1) : T(0);
}

// vec(rho) = e_idx: every element zero except element idx = 1 (rho = |r><c|, idx = r + c 2^n)
template <typename T>
__global__ void init_basis_kernel(T* __restrict__ rho, uint64_t nreal, uint64_t idx) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nreal; i += (uint64_t)gridDim.x * blockDim.x)
    rho[i] = (i == 2 * idx) ? T(1) : T(0);
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

// rho <- f rho in place: every element read once and written once with 16-byte accesses
// (one FP64 or two FP32 complex values per access), non-temporal (the data is not reused).
// Each workgroup owns one contiguous range of the state; the ranges of the workgroups that run
// on one XCD (workgroups are dealt round-robin over the 8 XCDs) are adjacent.  Each thread
// loads U accesses spaced one workgroup apart before it stores any of them, so a wave keeps U
// loads in flight.  This is the plain streaming kernel of the state buffer (one read and one
// write of every element, nothing else), so its rate is the bandwidth that an in-place pass
// over vec(rho) can reach.
template <typename V, typename S, int U>
__global__ __launch_bounds__(256) void scale_kernel(V* __restrict__ x, uint64_t nvec, S f) {
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t r = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;  // a bijection of [0, G)
  const uint64_t per = (nvec + G - 1) / G;
  const uint64_t lo = (uint64_t)r * per;
  const uint64_t hi = lo + per < nvec ? lo + per : nvec;
  for (uint64_t base = lo + threadIdx.x; base < hi; base += 256 * U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * 256;
      if (i < hi) v[u] = __builtin_nontemporal_load(x + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * 256;
      if (i < hi) __builtin_nontemporal_store(v[u] * f, x + i);
    }
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

// M <- S_op M for an operation on j = log4(DJ) <= 2 qubits: it mixes only the DJ rows of M that
// differ in its target bits, so each thread owns such groups of one column and rewrites them
// in place from registers.
template <int DJ>
__device__ inline void compose_groups(f64x2* M, const f64x2* Sl, const uint32_t* dep, int Dk, uint32_t tmask) {
  const uint32_t freemask = (uint32_t)(Dk - 1) & ~tmask;
  const int ngroups = Dk * (Dk / DJ);
  for (int gi = threadIdx.x; gi < ngroups; gi += blockDim.x) {
    const int c = gi % Dk;
    uint32_t a0 = 0, rb = (uint32_t)(gi / Dk);
    for (uint32_t m = freemask; m; m &= m - 1) {  // deposit rb into the non-target bits
      if (rb & 1u) a0 |= m & (0u - m);
      rb >>= 1;
    }
    f64x2 x[DJ];
#pragma unroll
    for (int b = 0; b < DJ; ++b) x[b] = M[(a0 | dep[b]) * Dk + c];
#pragma unroll 1
    for (int a = 0; a < DJ; ++a) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int b = 0; b < DJ; ++b) {
        const f64x2 w = Sl[a * DJ + b];
        sr += w[0] * x[b][0] - w[1] * x[b][1];
        si += w[0] * x[b][1] + w[1] * x[b][0];
      }
      M[(a0 | dep[a]) * Dk + c] = f64x2{sr, si};
    }
  }
}

// One workgroup per block: M <- S_op(embedded) M for each operation, starting from M = I.
// Column c of the result is vec of the block's action on the basis operator with vec
// index c, so the final M is S_blk = S_last ... S_first.  M stays in LDS (one buffer, updated
// in place).  Operations on one or two qubits update row groups in place (compose_groups);
// a three-qubit operation mixes whole columns, so each thread computes its outputs into
// registers (superoperator read from global memory) and writes them after a barrier.
template <int KMAX>
__global__ __launch_bounds__(256) void compose_kernel(const FuseBlockDev* __restrict__ blocks,
                                                      const FuseOpDev* __restrict__ ops,
                                                      const double* __restrict__ sops, double* __restrict__ out) {
  constexpr int DMAX = 1 << (2 * KMAX);
  constexpr int OUT_PER_THREAD = (DMAX * DMAX + 255) / 256;
  __shared__ f64x2 M[DMAX * DMAX];
  __shared__ f64x2 Sl[16 * 16];
  __shared__ uint32_t dep[64];
  const FuseBlockDev blk = blocks[blockIdx.x];
  const int k = blk.k, Dk = 1 << (2 * k);
  for (int e = threadIdx.x; e < Dk * Dk; e += blockDim.x) M[e] = f64x2{(e / Dk) == (e % Dk) ? 1.0 : 0.0, 0.0};
  for (int oi = 0; oi < blk.op_count; ++oi) {
    const FuseOpDev op = ops[blk.op_begin + oi];
    const int j = op.j, Dj = 1 << (2 * j);
    uint32_t tmask = 0;
    for (int t = 0; t < j; ++t) tmask |= (1u << op.pos[t]) | (1u << (k + op.pos[t]));
    __syncthreads();  // the previous operation's reads of Sl, dep and M are done
    const double* S = sops + 2 * op.sop_off;
    if (j <= 2)
      for (int e = threadIdx.x; e < Dj * Dj; e += blockDim.x) Sl[e] = f64x2{S[2 * e], S[2 * e + 1]};
    for (int b = threadIdx.x; b < Dj; b += blockDim.x) {
      uint32_t r = 0;
      for (int t = 0; t < j; ++t) {
        if ((b >> t) & 1) r |= 1u << op.pos[t];
        if ((b >> (j + t)) & 1) r |= 1u << (k + op.pos[t]);
      }
      dep[b] = r;
    }
    __syncthreads();
    if (j == 1) {
      compose_groups<4>(M, Sl, dep, Dk, tmask);
    } else if (j == 2) {
      compose_groups<16>(M, Sl, dep, Dk, tmask);
    } else {
      f64x2 y[OUT_PER_THREAD];
#pragma unroll
      for (int i = 0; i < OUT_PER_THREAD; ++i) {
        const int e = threadIdx.x + i * (int)blockDim.x;
        y[i] = f64x2{0.0, 0.0};
        if (e >= Dk * Dk) continue;
        const int a = e / Dk, c = e % Dk;
        uint32_t aloc = 0;
        for (int t = 0; t < j; ++t) {
          aloc |= (uint32_t)((a >> op.pos[t]) & 1) << t;
          aloc |= (uint32_t)((a >> (k + op.pos[t])) & 1) << (j + t);
        }
        const uint32_t abase = (uint32_t)a & ~tmask;
        double sr = 0.0, si = 0.0;
        for (int b = 0; b < Dj; ++b) {
          const double wr = S[2 * (aloc * Dj + b)], wi = S[2 * (aloc * Dj + b) + 1];
          const f64x2 v = M[(abase | dep[b]) * Dk + c];
          sr += wr * v[0] - wi * v[1];
          si += wr * v[1] + wi * v[0];
        }
        y[i] = f64x2{sr, si};
      }
      __syncthreads();  // every read of M is done before it is overwritten
#pragma unroll
      for (int i = 0; i < OUT_PER_THREAD; ++i) {
        const int e = threadIdx.x + i * (int)blockDim.x;
        if (e < Dk * Dk) M[e] = y[i];
      }
    }
  }
  __syncthreads();
  double* O = out + 2 * blk.out_off;
  for (int e = threadIdx.x; e < Dk * Dk; e += blockDim.x) {
    O[2 * e] = M[e][0];
    O[2 * e + 1] = M[e][1];
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

template <typename TA, typename TB>
__global__ __launch_bounds__(RED_THREADS) void compare_kernel(const TA* __restrict__ a, const TB* __restrict__ b,
                                                             uint64_t nel, double* __restrict__ partials) {
  __shared__ double sh[RED_THREADS / 64];
  double dd = 0.0, mx = 0.0, aa = 0.0;
  for (uint64_t e = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; e < nel; e += (uint64_t)gridDim.x * RED_THREADS) {
    const double ar = (double)a[2 * e], ai = (double)a[2 * e + 1];
    const double dr = ar - (double)b[2 * e], di = ai - (double)b[2 * e + 1];
    const double d2 = dr * dr + di * di;
    dd += d2;
    mx = d2 > mx ? d2 : mx;
    aa += ar * ar + ai * ai;
  }
  const double t0 = block_sum(dd, sh);
  const double t2 = block_sum(aa, sh);
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_down(mx, o, 64);
    mx = other > mx ? other : mx;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) m = sh[i] > m ? sh[i] : m;
    partials[blockIdx.x] = t0;
    partials[gridDim.x + blockIdx.x] = m;
    partials[2 * gridDim.x + blockIdx.x] = t2;
  }
}

__global__ void compare_finish_kernel(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s0 = 0.0, m = 0.0, s2 = 0.0;
    for (int i = 0; i < nb; ++i) {
      s0 += partials[i];
      m = partials[nb + i] > m ? partials[nb + i] : m;
      s2 += partials[2 * nb + i];
    }
    out[0] = sqrt(s0);
    out[1] = sqrt(m);
    out[2] = sqrt(s2);
  }
}

// Reduced density matrix on the kept qubits: out[a][b] = sum over the other qubits' values f
// of rho[dep(a) | f][dep(b) | f].  One workgroup per output element (a, b); FP64.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void reduced_kernel(const T* __restrict__ rho, int n, int k,
                                                             const int* __restrict__ keep,
                                                             double* __restrict__ out) {
  __shared__ double sh[RED_THREADS / 64];
  __shared__ int kq[8];
  if (threadIdx.x < (unsigned)k) kq[threadIdx.x] = keep[threadIdx.x];
  __syncthreads();
  const int D = 1 << k;
  const int a = blockIdx.x % D, b = blockIdx.x / D;
  uint64_t ra = 0, rb = 0, kmask = 0;
  for (int t = 0; t < k; ++t) {
    kmask |= 1ull << kq[t];
    if ((a >> t) & 1) ra |= 1ull << kq[t];
    if ((b >> t) & 1) rb |= 1ull << kq[t];
  }
  const uint64_t nf = 1ull << (n - k);
  double sr = 0.0, si = 0.0;
  for (uint64_t f = threadIdx.x; f < nf; f += RED_THREADS) {
    // deposit f into the bits outside kmask
    uint64_t x = 0, ff = f;
    for (int bit = 0; bit < n; ++bit)
      if (!((kmask >> bit) & 1ull)) {
        x |= (ff & 1ull) << bit;
        ff >>= 1;
      }
    const uint64_t e = (ra | x) + ((rb | x) << n);
    sr += (double)rho[2 * e];
    si += (double)rho[2 * e + 1];
  }
  const double tr = block_sum(sr, sh);
  const double ti = block_sum(si, sh);
  if (threadIdx.x == 0) {
    out[2 * (a * D + b)] = tr;
    out[2 * (a * D + b) + 1] = ti;
  }
}

// ------------------------------------------------------------------------------------
// readout error and sampling (FP64, on the probability vector)
// ------------------------------------------------------------------------------------

// Qubit t is read as 1 when it is 0 with probability p10 and as 0 when it is 1 with p01:
// q[x with bit t = 0] = (1 - p10) p[.0.] + p01 p[.1.],  q[.1.] = p10 p[.0.] + (1 - p01) p[.1.]
__global__ void readout_kernel(double* __restrict__ p, uint64_t dim, int t, double p01, double p10) {
  const uint64_t half = dim >> 1, bit = 1ull << t, low = bit - 1ull;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x0 = ((i & ~low) << 1) | (i & low), x1 = x0 | bit;
    const double a = p[x0], b = p[x1];
    p[x0] = (1.0 - p10) * a + p01 * b;
    p[x1] = p10 * a + (1.0 - p01) * b;
  }
}

// Inclusive prefix sums of p[0..dim) by one workgroup of 1024 threads (fixed order).
__global__ __launch_bounds__(1024) void cdf_kernel(const double* __restrict__ p, uint64_t dim, double* __restrict__ cdf) {
  __shared__ double part[1024];
  const uint64_t per = (dim + 1023) / 1024;
  const uint64_t b = threadIdx.x * per, e = (b + per < dim) ? b + per : dim;
  double s = 0.0;
  for (uint64_t x = b; x < e; ++x) s += p[x];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int i = 0; i < 1024; ++i) {
      const double v = part[i];
      part[i] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = part[threadIdx.x];
  for (uint64_t x = b; x < e; ++x) {
    run += p[x];
    cdf[x] = run;
  }
}

// Shot i draws u = top 53 bits of SplitMix64((seed << 40) + i) in [0, 1) and returns the
// smallest x with cdf[x] > u * cdf[dim - 1].
__global__ void sample_kernel(const double* __restrict__ cdf, uint64_t dim, uint64_t shots, uint64_t seed,
                              uint64_t* __restrict__ out) {
  const double total = cdf[dim - 1];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < shots; i += (uint64_t)gridDim.x * blockDim.x) {
    const double u = (double)(splitmix64((seed << 40) + i) >> 11) * 0x1.0p-53 * total;
    uint64_t lo = 0, hi = dim - 1;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (cdf[mid] > u) hi = mid;
      else lo = mid + 1;
    }
    out[i] = lo;
  }
}

// ------------------------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------------------------

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

// The matrix units' sustained rate in the multiplication loop of the pass kernels, without
// the loop's LDS traffic, barriers or memory: one workgroup of eight waves per CU (two per
// SIMD, as the pass kernels' consumer waves), each wave repeating two column blocks of three
// independent 16x16x4 accumulation chains over four k-steps with register operands, followed
// by the 3M combination on the vector ALU.  Operands change every iteration so nothing is
// hoisted; one store per thread at the end keeps the work.
template <typename T, typename A>
__global__ __launch_bounds__(512) void mfma_rate_kernel(T* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  T a[12], b[8][2];
#pragma unroll
  for (int i = 0; i < 12; ++i) a[i] = T(1) + T(1e-7) * (T)(lane + i);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    b[i][0] = T(1e-7) * (T)i;
    b[i][1] = T(2e-7) * (T)i;
  }
  A keep = {0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      A p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T br = b[blk * 4 + s][0], bi = b[blk * 4 + s][1];
        if constexpr (sizeof(T) == 8) {
          p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3 * s], br, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3 * s + 1], bi, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3 * s + 2], br + bi, p3, 0, 0, 0);
        } else {
          p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3 * s], br, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3 * s + 1], bi, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3 * s + 2], br + bi, p3, 0, 0, 0);
        }
      }
      keep += (p1 - p2) + (p3 - p1 - p2);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      b[i][0] += T(1e-9);
      b[i][1] -= T(1e-9);
    }
  }
  out[(size_t)blockIdx.x * 512 + threadIdx.x] = keep[0] + keep[1] + keep[2] + keep[3];
}

double mfma_rate_tflops(tanq_prec p) {
  constexpr int kIters = 8192;
  const int cus = device_cu_count();
  const size_t bytes = (size_t)cus * 512 * (p == TANQ_F64 ? 8 : 4);
  void* out = nullptr;
  TANQ_HIP(hipMalloc(&out, bytes));
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 0.f;
  try {
    TANQ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    TANQ_HIP(hipEventCreate(&e0));
    TANQ_HIP(hipEventCreate(&e1));
    for (int rep = 0; rep < 4; ++rep) {  // the first launch warms the clocks up; keep the fastest
      TANQ_HIP(hipEventRecord(e0, s));
      if (p == TANQ_F64)
        hipLaunchKernelGGL((mfma_rate_kernel<double, f64x4>), dim3(cus), dim3(512), 0, s, (double*)out, kIters);
      else
        hipLaunchKernelGGL((mfma_rate_kernel<float, f32x4>), dim3(cus), dim3(512), 0, s, (float*)out, kIters);
      TANQ_HIP(hipGetLastError());
      TANQ_HIP(hipEventRecord(e1, s));
      TANQ_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      TANQ_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0 && (best == 0.f || ms < best)) best = ms;
    }
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(out);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  TANQ_HIP(hipFree(out));
  // 8 waves x 24 products of 16 x 16 x 4 (2048 flops each) per iteration
  const double flops = (double)cus * 8.0 * kIters * 24.0 * 2048.0;
  return flops / (best * 1e-3) / 1e12;
}

void launch_scale(void* rho, int n, tanq_prec p, double f, hipStream_t s) {
  constexpr int U = 4;
  // 16-byte accesses: one FP64 complex element, or two FP32 ones
  const uint64_t nvec = (p == TANQ_F64) ? (1ull << (2 * n)) : (1ull << (2 * n)) / 2;
  uint64_t blocks = (nvec + 256 * U - 1) / (256 * U);
  const uint64_t cap = (uint64_t)device_cu_count() * 32;
  if (blocks > cap) blocks = cap;
  if (p == TANQ_F64)
    hipLaunchKernelGGL((scale_kernel<f64x2, double, U>), dim3((unsigned)blocks), dim3(256), 0, s, (f64x2*)rho,
                       nvec, f);
  else
    hipLaunchKernelGGL((scale_kernel<f32x4, float, U>), dim3((unsigned)blocks), dim3(256), 0, s, (f32x4*)rho,
                       nvec, (float)f);
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

void launch_init_basis(void* rho, int n, tanq_prec p, uint64_t idx, hipStream_t s) {
  const uint64_t nreal = 2ull << (2 * n);
  uint64_t blocks = (nreal + 255) / 256;
  const uint64_t cap = (uint64_t)device_cu_count() * 64;
  if (blocks > cap) blocks = cap;
  if (p == TANQ_F64)
    hipLaunchKernelGGL(init_basis_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)rho, nreal, idx);
  else
    hipLaunchKernelGGL(init_basis_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)rho, nreal, idx);
  TANQ_HIP(hipGetLastError());
}

void launch_reduced(const void* rho, int n, tanq_prec p, int k, const int* keep_dev, double* out_dev, hipStream_t s) {
  const unsigned nb = 1u << (2 * k);
  if (p == TANQ_F64)
    hipLaunchKernelGGL(reduced_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, s, (const double*)rho, n, k, keep_dev,
                       out_dev);
  else
    hipLaunchKernelGGL(reduced_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, s, (const float*)rho, n, k, keep_dev,
                       out_dev);
  TANQ_HIP(hipGetLastError());
}

void launch_readout(double* probs_dev, int n, const double* p01, const double* p10, hipStream_t s) {
  const uint64_t dim = 1ull << n;
  uint64_t blocks = (dim / 2 + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  for (int t = 0; t < n; ++t) {
    hipLaunchKernelGGL(readout_kernel, dim3((unsigned)blocks), dim3(256), 0, s, probs_dev, dim, t, p01[t], p10[t]);
    TANQ_HIP(hipGetLastError());
  }
}

void launch_sample(const double* probs_dev, int n, double* cdf_dev, uint64_t shots, uint64_t seed, uint64_t* out_dev,
                   hipStream_t s) {
  const uint64_t dim = 1ull << n;
  hipLaunchKernelGGL(cdf_kernel, dim3(1), dim3(1024), 0, s, probs_dev, dim, cdf_dev);
  TANQ_HIP(hipGetLastError());
  uint64_t blocks = (shots + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(256), 0, s, cdf_dev, dim, shots, seed, out_dev);
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

template <typename TA, typename TB>
static void compare_typed(const void* a, const void* b, uint64_t nel, int nb, double* partials, hipStream_t s) {
  hipLaunchKernelGGL((compare_kernel<TA, TB>), dim3(nb), dim3(RED_THREADS), 0, s, (const TA*)a, (const TB*)b, nel,
                     partials);
}

void launch_compare(const void* a, tanq_prec pa, const void* b, tanq_prec pb, uint64_t nel, double* partials,
                    double* result_dev, hipStream_t s) {
  const int nb = red_blocks(nel);
  if (pa == TANQ_F64 && pb == TANQ_F64) compare_typed<double, double>(a, b, nel, nb, partials, s);
  else if (pa == TANQ_F64) compare_typed<double, float>(a, b, nel, nb, partials, s);
  else if (pb == TANQ_F64) compare_typed<float, double>(a, b, nel, nb, partials, s);
  else compare_typed<float, float>(a, b, nel, nb, partials, s);
  TANQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(compare_finish_kernel, dim3(1), dim3(64), 0, s, partials, nb, result_dev);
  TANQ_HIP(hipGetLastError());
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
