// Host side of the multi-superoperator passes: the process-wide pass limit and the geometry of
// one pass (tile bits, runs of fixed bits, per-superoperator tile offsets and the LDS swizzle,
// which a seeded search picks so that each superoperator's MFMA accesses avoid bank conflicts).
// The kernels are in pass.hip.
#include <algorithm>
#include <atomic>
#include <cstring>

#include "internal.hpp"

namespace tanq {

int pass_tile_bits(tanq_prec p) { return p == TANQ_F64 ? kPassTileBitsF64 : kPassTileBitsF32; }
int pass_max(tanq_prec p) { return p == TANQ_F64 ? kPassMaxF64 : kPassMaxF32; }

static std::atomic<int> g_pass_limit{kPassMax};
int pass_limit() { return g_pass_limit.load(); }
void set_pass_limit(int m) {
  if (m < 1 || m > kPassMax) fail(TANQ_E_ARG, "pass limit must be 1..8");
  g_pass_limit.store(m);
}

// ------------------------------------------------------------------------------------
// host: geometry and swizzle of one pass
// ------------------------------------------------------------------------------------

namespace {

int gf2_rank(uint32_t* v, int cnt) {
  int r = 0;
  for (int bit = 31; bit >= 0 && r < cnt; --bit) {
    int piv = -1;
    for (int i = r; i < cnt; ++i)
      if ((v[i] >> bit) & 1u) {
        piv = i;
        break;
      }
    if (piv < 0) continue;
    std::swap(v[r], v[piv]);
    for (int i = 0; i < cnt; ++i)
      if (i != r && ((v[i] >> bit) & 1u)) v[i] ^= v[r];
    ++r;
  }
  return r;
}

struct SwzProblem {
  int W, V, m;
  uint32_t fbits[kPassMax][4];  // lowest four free tile bits of each superoperator
  uint32_t t1[kPassMax], t2[kPassMax];
};

uint32_t low_of(uint32_t x, const uint8_t* xcol, int W) {
  uint32_t r = x & ((1u << W) - 1u);
  for (int b = W; b < 16; ++b)
    if ((x >> b) & 1u) r ^= xcol[b];
  return r;
}

// Number of bank-conflict-free access patterns under xcol (2 per superoperator).
int swz_score(const SwzProblem& P, const uint8_t* xcol) {
  int score = 0;
  for (int j = 0; j < P.m; ++j) {
    uint32_t v[5];
    if (P.W == 4) {
      for (int q = 0; q < 4; ++q) v[q] = low_of(1u << P.fbits[j][q], xcol, 4);
      score += 2 * (gf2_rank(v, 4) == 4);
    } else {
      for (int q = 0; q < 4; ++q) v[q] = low_of(1u << P.fbits[j][q], xcol, 5);
      v[4] = low_of(P.t1[j], xcol, 5);
      score += gf2_rank(v, 5) == 5;
      for (int q = 0; q < 4; ++q) v[q] = low_of(1u << P.fbits[j][q], xcol, 5);
      v[4] = low_of(P.t2[j], xcol, 5);
      score += gf2_rank(v, 5) == 5;
    }
  }
  return score;
}

// Upper bound of swz_score over all swizzles: a pattern's vectors from bits inside the window
// are fixed unit vectors; those from bits above it can be any vectors of the allowed columns
// (FP32 columns never set bit 0, so an FP32 pattern spans bit 0 only through tile bit 0).
int swz_bound(const SwzProblem& P) {
  auto ok = [&](const uint32_t* bits, int cnt) {
    uint32_t fixed = 0;
    int above = 0;
    for (int q = 0; q < cnt; ++q) {
      if (bits[q] < (uint32_t)P.W) {
        if ((fixed >> bits[q]) & 1u) return false;  // a repeated unit vector
        fixed |= 1u << bits[q];
      } else {
        ++above;
      }
    }
    if (P.W == 5) return (fixed & 1u) && above <= 4 - __builtin_popcount(fixed & ~1u);
    return above <= P.W - __builtin_popcount(fixed);
  };
  int b = 0;
  for (int j = 0; j < P.m; ++j) {
    uint32_t v[5];
    for (int q = 0; q < 4; ++q) v[q] = P.fbits[j][q];
    if (P.W == 4) {
      b += 2 * ok(v, 4);
    } else {
      v[4] = (uint32_t)__builtin_ctz(P.t1[j]);
      b += ok(v, 5);
      v[4] = (uint32_t)__builtin_ctz(P.t2[j]);
      b += ok(v, 5);
    }
  }
  return b;
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

PassGeom make_pass_geom(int n, int m, const int* qubits, const uint32_t* op_off, tanq_prec p, int* conflict_free,
                        int* achievable) {
  if (m < 1 || m > kPassMax) fail(TANQ_E_ARG, "pass length outside 1..kPassMax");
  PassGeom g;
  std::memset(&g, 0, sizeof(g));
  const int nb = 2 * n;
  const int V = pass_tile_bits(p);
  if (nb < V) fail(TANQ_E_ARG, "state too small for a pass tile");
  uint64_t vmask = 0;
  for (int j = 0; j < m; ++j)
    for (int t = 0; t < 2; ++t) {
      const int q = qubits[2 * j + t];
      if (q < 0 || q >= n) fail(TANQ_E_ARG, "pass qubit out of range");
      vmask |= (1ull << q) | (1ull << (q + n));
    }
  if (__builtin_popcountll(vmask) > V) fail(TANQ_E_ARG, "pass qubits do not fit one tile");
  for (int b = 0, need = V - __builtin_popcountll(vmask); b < nb && need > 0; ++b)
    if (!((vmask >> b) & 1ull)) {
      vmask |= 1ull << b;
      --need;
    }
  int cnt = 0;
  int local_of[64];
  for (int b = 0; b < nb; ++b) {
    local_of[b] = -1;
    if ((vmask >> b) & 1ull) {
      local_of[b] = cnt;
      g.vpos[cnt++] = (uint8_t)b;
    }
  }
  if (cnt != V) fail(TANQ_E_STATE, "pass tile bit count");
  // FP32 moves two elements per 16-byte slot: global bit 0 must be tile bit 0
  if (p != TANQ_F64 && g.vpos[0] != 0) fail(TANQ_E_STATE, "pass tile without global bit 0");
  g.V = V;
  g.m = m;

  uint32_t tj[kPassMax][16];
  SwzProblem P{};
  P.W = (p == TANQ_F64) ? 4 : 5;
  P.V = V;
  P.m = m;
  for (int j = 0; j < m; ++j) {
    const int tgt[4] = {qubits[2 * j], qubits[2 * j + 1], qubits[2 * j] + n, qubits[2 * j + 1] + n};
    uint32_t tmask = 0;
    int tpos[4];
    for (int t = 0; t < 4; ++t) {
      tpos[t] = local_of[tgt[t]];
      tmask |= 1u << tpos[t];
    }
    if (__builtin_popcount(tmask) != 4) fail(TANQ_E_ARG, "a pass superoperator repeats a qubit");
    for (int l = 0; l < 16; ++l) {
      uint32_t r = 0;
      for (int t = 0; t < 4; ++t)
        if ((l >> t) & 1) r |= 1u << tpos[t];
      tj[j][l] = r;
    }
    g.free_mask[j] = ((1u << V) - 1u) & ~tmask;
    g.op_off[j] = op_off[j];
    int q = 0;
    for (int b = 0; b < V && q < 4; ++b)
      if ((g.free_mask[j] >> b) & 1u) P.fbits[j][q++] = (uint32_t)b;
    P.t1[j] = tj[j][1];  // FP32 operand reads: lanes 0-31 cover rows 0 and 1
    P.t2[j] = tj[j][4];  // FP32 result writes: lanes 0-31 cover rows 0-3 and 4-7
  }

  // swizzle: the identity first, then seeded random candidates, keeping the best (reaching the
  // bound ends the search)
  uint8_t best[16] = {0};
  int best_score = swz_score(P, best);
  const int perfect = swz_bound(P);
  uint64_t seed = 0x7A3Cull ^ ((uint64_t)n << 32) ^ (uint64_t)m;
  // FP32 columns never set bit 0: a 16-byte slot's two elements keep their order, as the
  // global-to-LDS loads require
  const uint32_t wmask = ((1u << P.W) - 1u) & (p == TANQ_F64 ? ~0u : ~1u);
  for (int trial = 0; trial < 4000 && best_score < perfect; ++trial) {
    uint8_t cand[16] = {0};
    const uint64_t r0 = splitmix(seed), r1 = splitmix(seed);
    for (int b = P.W; b < V; ++b) {
      const uint64_t r = (b < 8 + P.W) ? (r0 >> (8 * (b - P.W))) : (r1 >> (8 * (b - P.W - 8)));
      cand[b] = (uint8_t)((uint32_t)r & wmask);
    }
    const int sc = swz_score(P, cand);
    if (sc > best_score) {
      best_score = sc;
      std::memcpy(best, cand, sizeof(best));
    }
  }
  std::memcpy(g.xcol, best, sizeof(best));
  if (conflict_free) *conflict_free = best_score;
  if (achievable) *achievable = perfect;
  auto S = [&](uint32_t e) {
    uint32_t x = e;
    for (int b = P.W; b < 16; ++b)
      if ((e >> b) & 1u) x ^= g.xcol[b];
    return x;
  };
  for (int j = 0; j < m; ++j)
    for (int l = 0; l < 16; ++l) g.stj[j][l] = S(tj[j][l]);
  // S(e) = e ^ X(e) with X linear in the bits above the window and valued inside it, so S is an
  // involution of [0, 2^V) exactly when every column lies inside the window (and, in FP32, never
  // flips bit 0, which keeps slot pairs whole and in order); columns of bits >= V are unused
  for (int b = 0; b < 16; ++b)
    if ((b < P.W && g.xcol[b]) || (g.xcol[b] >> P.W) || (b >= V && g.xcol[b]) || (p != TANQ_F64 && (g.xcol[b] & 1u)))
      fail(TANQ_E_STATE, "pass swizzle column outside the bank window");

  // runs of fixed bits: the maximal runs of global bits outside the tile, lowest first, each
  // taking the next tile-index bits; so a tile's base is the tile index deposited into those
  // bits, which the FP64 pass kernel relies on to step from one tile's base to the next
  int src = 0, nr = 0;
  for (int b = 0; b < nb;) {
    if ((vmask >> b) & 1ull) {
      ++b;
      continue;
    }
    int e = b;
    while (e < nb && !((vmask >> e) & 1ull)) ++e;
    if (nr >= 16) fail(TANQ_E_STATE, "too many runs of fixed bits");
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

// Specialised-wave shape: 640 threads, 2 producer and 8 consumer waves.
}  // namespace tanq
