// C ABI of libtanq (declared in include/tanq.h): handles, circuits, fusion and
// measurement entry points.  Every compute step runs in the HIP kernels of kernels.hip;
// this file validates arguments, owns memory and orders work on the handle's stream.
#include <complex>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "abi_util.hpp"
#include "circuit.hpp"

using namespace tanq;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace tanq {
tanq_status set_last_error(tanq_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
void clear_last_error() { g_last_error.clear(); }
}  // namespace tanq

namespace {

tanq_status set_error(tanq_status code, const std::string& msg) { return set_last_error(code, msg); }

constexpr int MAX_N = 17;
constexpr int RING = 8;
constexpr size_t SLOT_DOUBLES = 2 * 64 * 64;  // one 3-qubit superoperator, complex128

void check_prec(tanq_prec p) {
  if (p != TANQ_F64 && p != TANQ_F32) fail(TANQ_E_ARG, "precision must be TANQ_F64 or TANQ_F32");
}

void check_qubits(int n, int k, const int* q, int kmax) {
  if (k < 1 || k > kmax) fail(TANQ_E_ARG, "width must be in 1.." + std::to_string(kmax));
  if (k > n) fail(TANQ_E_ARG, "width exceeds the number of qubits");
  if (!q) fail(TANQ_E_ARG, "qubits is NULL");
  for (int t = 0; t < k; ++t) {
    if (q[t] < 0 || q[t] >= n) fail(TANQ_E_ARG, "qubit " + std::to_string(q[t]) + " out of range");
    for (int u = 0; u < t; ++u)
      if (q[u] == q[t]) fail(TANQ_E_ARG, "duplicate qubit " + std::to_string(q[t]));
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    TANQ_HIP(hipGetDevice(&prev));
    if (prev != dev) TANQ_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

struct tanq_dm_s {
  int n = 0;
  tanq_prec prec = TANQ_F64;
  void* ptr = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  double* probs_dev = nullptr;
  double* partials = nullptr;
  double* result_dev = nullptr;
  uint64_t* masks_dev = nullptr;
  double* s_raw_dev = nullptr;      // RING slots of a FP64 superoperator
  unsigned char* s_packed_dev = nullptr;  // RING slots of a packed operand
  double* pinned = nullptr;         // RING slots, host
  hipEvent_t ev[RING] = {};
  int ring = 0;

  uint64_t elements() const { return 1ull << (2 * n); }
  size_t bytes() const { return (size_t)elements() * elem_size(prec); }
};

struct tanq_fused_s {
  int n = 0;
  tanq_prec prec = TANQ_F64;
  int mode = 0;
  int device = 0;
  int source_ops = 0;
  int count_k[4] = {0, 0, 0, 0};
  std::vector<FusedBlockHost> blocks;
  double* raw = nullptr;
  unsigned char* packed = nullptr;
  // pass geometries already built, by (first block, length)
  std::mutex pass_mu;
  std::map<std::pair<int, int>, tanq::PassGeom> passes;
};

namespace {

void dm_alloc_scratch(tanq_dm_s* d) {
  const uint64_t dim = 1ull << d->n;
  TANQ_HIP(hipMalloc((void**)&d->probs_dev, dim * sizeof(double)));
  TANQ_HIP(hipMalloc((void**)&d->partials, (size_t)reduce_partials() * sizeof(double)));
  TANQ_HIP(hipMalloc((void**)&d->result_dev, 4096 * sizeof(double)));
  TANQ_HIP(hipMalloc((void**)&d->masks_dev, 3 * 2048 * sizeof(uint64_t)));
  TANQ_HIP(hipMalloc((void**)&d->s_raw_dev, RING * SLOT_DOUBLES * sizeof(double)));
  TANQ_HIP(hipMalloc((void**)&d->s_packed_dev, RING * packed_bytes(3, TANQ_F64)));
  TANQ_HIP(hipHostMalloc((void**)&d->pinned, RING * SLOT_DOUBLES * sizeof(double), hipHostMallocDefault));
  for (int i = 0; i < RING; ++i) TANQ_HIP(hipEventCreateWithFlags(&d->ev[i], hipEventDisableTiming));
}

void dm_release(tanq_dm_s* d) {
  if (!d) return;
  (void)hipSetDevice(d->device);
  (void)hipStreamSynchronize(d->stream);
  for (int i = 0; i < RING; ++i)
    if (d->ev[i]) (void)hipEventDestroy(d->ev[i]);
  if (d->pinned) (void)hipHostFree(d->pinned);
  dfree(d->probs_dev);
  dfree(d->partials);
  dfree(d->result_dev);
  dfree(d->masks_dev);
  dfree(d->s_raw_dev);
  dfree(d->s_packed_dev);
  if (d->owned && d->ptr) (void)hipFree(d->ptr);
  delete d;
}

tanq_dm_s* dm_new(int n, tanq_prec p, void* stream) {
  if (n < 1 || n > MAX_N) fail(TANQ_E_ARG, "n must be in 1..17");
  check_prec(p);
  std::unique_ptr<tanq_dm_s> d(new tanq_dm_s);
  d->n = n;
  d->prec = p;
  d->stream = (hipStream_t)stream;
  TANQ_HIP(hipGetDevice(&d->device));
  return d.release();
}

void check_dm(tanq_dm d) {
  if (!d) fail(TANQ_E_ARG, "density-matrix handle is NULL");
}

void parse_pauli(int n, const char* s, uint64_t out[3]) {
  if (!s) fail(TANQ_E_ARG, "Pauli string is NULL");
  uint64_t xm = 0, zm = 0;
  int ny = 0;
  int t = 0;
  for (; s[t] != '\0'; ++t) {
    if (t >= n) fail(TANQ_E_ARG, "Pauli string longer than n");
    switch (s[t]) {
      case 'I': break;
      case 'X': xm |= 1ull << t; break;
      case 'Y': xm |= 1ull << t; zm |= 1ull << t; ++ny; break;
      case 'Z': zm |= 1ull << t; break;
      default: fail(TANQ_E_ARG, std::string("bad Pauli character '") + s[t] + "'");
    }
  }
  if (t != n) fail(TANQ_E_ARG, "Pauli string must have exactly n characters");
  out[0] = xm;
  out[1] = zm;
  out[2] = (uint64_t)(ny & 3);
}

}  // namespace

constexpr int kPassMinTileBits = 8;  // passes need at least 2^8 tiles (one per CU)

// Contiguous elements (log2) of a pass tile in vec(rho): the tile holds the row and column bit
// of every qubit in `qmask` plus the lowest other bits up to V; the low run is the number of
// consecutive held bits from bit 0.  -1 if the qubits do not fit.
inline int pass_low_run(uint64_t qmask, int n, int V) {
  uint64_t held = qmask | (qmask << n);
  int fill = V - __builtin_popcountll(held);
  if (fill < 0) return -1;
  for (int b = 0; b < 2 * n && fill > 0; ++b)
    if (!((held >> b) & 1ull)) {
      held |= 1ull << b;
      --fill;
    }
  int c = 0;
  while (c < 2 * n && ((held >> c) & 1ull)) ++c;
  return c;
}

// Length of the pass that starts at block i (blocks before `end`): the longest run of
// consecutive 2-qubit blocks, at most `lim`, whose qubits fit one pass tile with runs of at
// least 128 contiguous bytes in vec(rho) (whole cache lines: shorter runs make the HBM fetch
// more than it uses); 1 when no pass applies (a different width, too small a state, passes
// switched off).  at(j, &q) returns the width of block j and points q at its qubits.
template <typename BlockAt>
int pass_run(BlockAt at, int i, int end, int n, tanq_prec p, int lim) {
  const int V = pass_tile_bits(p);
  const int min_run = p == TANQ_F64 ? 3 : 4;  // 8 x 16 B or 16 x 8 B
  lim = std::min(lim, pass_max(p));
  // smaller states (fewer pass tiles than CUs) are bound by launch and set-up costs, where
  // single applies with their smaller tiles do better
  if (lim < 2 || 2 * n - V < kPassMinTileBits) return 1;
  const int* q = nullptr;
  if (at(i, &q) != 2) return 1;
  uint64_t mask = (1ull << q[0]) | (1ull << q[1]);
  int m = 1;
  while (i + m < end && m < lim) {
    if (at(i + m, &q) != 2) break;
    const uint64_t nm = mask | (1ull << q[0]) | (1ull << q[1]);
    if (pass_low_run(nm, n, V) < min_run) break;
    mask = nm;
    ++m;
  }
  return m;
}

// Reorder a block list so that blocks that can share a pass are adjacent.  The first block not
// yet placed heads a pass.  A scan over the following blocks (within a short window) takes each
// 1- or 2-qubit block that fits the pass tile and commutes with every block it moves ahead of
// (shares no qubit with the blocks skipped so far); a skipped block blocks its qubits for the
// rest of the scan.  The pass's second member decides which blocks fit later, so the scan is
// repeated with each fitting block forced as the second member and the longest pass is kept.
// Taken blocks keep their relative order.  One-qubit members of a pass are widened to two
// qubits (the identity on a qubit the pass already holds), since a pass applies 2-qubit
// superoperators.  Reordering commuting superoperators leaves the product unchanged.  Returns
// the list unchanged where passes do not apply.
std::vector<PlanBlock> pass_order(const std::vector<PlanBlock>& pl, int n, tanq_prec p, int lim) {
  const int V = pass_tile_bits(p);
  const int min_run = p == TANQ_F64 ? 3 : 4;
  constexpr size_t kWindow = 16;
  lim = std::min(lim, pass_max(p));
  if (lim < 2 || 2 * n - V < kPassMinTileBits) return pl;
  auto qmask = [&](int b) {
    uint64_t m = 0;
    for (int q : pl[b].qubits) m |= 1ull << q;
    return m;
  };
  // blocks not yet placed; taken blocks lie within the window at the front, where a deque
  // erases in constant time
  std::deque<int> rem(pl.size());
  for (size_t i = 0; i < rem.size(); ++i) rem[i] = (int)i;
  auto fits = [&](int b, uint64_t U, uint64_t blocked) {
    const uint64_t qb = qmask(b);
    return pl[b].qubits.size() <= 2 && !(qb & blocked) && pass_low_run(U | qb, n, V) >= min_run;
  };
  // scan positions after `from`, starting from pass qubits U, taken positions `take` and
  // blocked qubits; returns the taken positions (increasing) and their qubit union
  auto scan = [&](size_t from, uint64_t U, uint64_t blocked, std::vector<size_t> take, uint64_t* Uout) {
    const size_t end = std::min(rem.size(), kWindow);
    for (size_t pos = from; pos < end && (int)take.size() < lim; ++pos) {
      const int b = rem[pos];
      if (fits(b, U, blocked)) {
        take.push_back(pos);
        U |= qmask(b);
      } else {
        blocked |= qmask(b);
      }
    }
    *Uout = U;
    return take;
  };
  std::vector<PlanBlock> out;
  out.reserve(pl.size());
  while (!rem.empty()) {
    const int b0 = rem[0];
    std::vector<size_t> take(1, 0);
    uint64_t U = qmask(b0);
    if (pl[b0].qubits.size() <= 2) {
      uint64_t Ub = 0;
      take = scan(1, U, 0, take, &Ub);
      U = Ub;
      // the same scan with each fitting block forced as the second member
      uint64_t blocked = 0;
      for (size_t pos = 1; pos < std::min(rem.size(), kWindow) && lim >= 3; ++pos) {
        const int b = rem[pos];
        if (fits(b, qmask(b0), blocked)) {
          uint64_t Uf = 0;
          std::vector<size_t> t = scan(pos + 1, qmask(b0) | qmask(b), blocked, std::vector<size_t>{0, pos}, &Uf);
          if (t.size() > take.size()) {
            take = std::move(t);
            U = Uf;
          }
        }
        blocked |= qmask(b);
      }
    }
    const bool pass = take.size() >= 2 && __builtin_popcountll(U) >= 2;
    for (size_t t : take) {
      PlanBlock b = pl[rem[t]];
      if (pass && b.qubits.size() == 1) {
        const int q = b.qubits[0];
        const uint64_t others = U & ~(1ull << q);
        b.qubits.push_back(__builtin_ctzll(others));
        std::sort(b.qubits.begin(), b.qubits.end());
      }
      out.push_back(std::move(b));
    }
    for (auto it = take.rbegin(); it != take.rend(); ++it) rem.erase(rem.begin() + (ptrdiff_t)*it);
  }
  return out;
}

extern "C" {

const char* tanq_last_error(void) { return g_last_error.c_str(); }

int tanq_version(void) { return 100; }

tanq_status tanq_dm_init(int n, tanq_prec p, void* hip_stream, tanq_dm* out) {
  return guarded([&] {
    if (!out) fail(TANQ_E_ARG, "out is NULL");
    *out = nullptr;
    tanq_dm_s* d = dm_new(n, p, hip_stream);
    try {
      size_t free_b = 0, total_b = 0;
      TANQ_HIP(hipMemGetInfo(&free_b, &total_b));
      if (d->bytes() + (64ull << 20) > free_b)
        fail(TANQ_E_OOM, "density matrix needs " + std::to_string(d->bytes()) + " bytes, " +
                             std::to_string(free_b) + " free");
      hipError_t e = hipMalloc(&d->ptr, d->bytes());
      if (e != hipSuccess) fail(TANQ_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
      d->owned = true;
      dm_alloc_scratch(d);
      launch_init_zero(d->ptr, n, p, d->stream);
    } catch (...) {
      dm_release(d);
      throw;
    }
    *out = d;
  });
}

tanq_status tanq_dm_wrap(int n, tanq_prec p, void* dev_ptr, void* hip_stream, tanq_dm* out) {
  return guarded([&] {
    if (!out) fail(TANQ_E_ARG, "out is NULL");
    *out = nullptr;
    if (!dev_ptr) fail(TANQ_E_ARG, "device pointer is NULL");
    if (((uintptr_t)dev_ptr) & 15u) fail(TANQ_E_ARG, "device pointer must be 16-byte aligned");
    tanq_dm_s* d = dm_new(n, p, hip_stream);
    try {
      d->ptr = dev_ptr;
      d->owned = false;
      dm_alloc_scratch(d);
    } catch (...) {
      dm_release(d);
      throw;
    }
    *out = d;
  });
}

tanq_status tanq_dm_free(tanq_dm d) {
  return guarded([&] { dm_release(d); });
}

tanq_status tanq_dm_reset(tanq_dm d) {
  return guarded([&] {
    check_dm(d);
    DeviceGuard g(d->device);
    launch_init_zero(d->ptr, d->n, d->prec, d->stream);
  });
}

tanq_status tanq_dm_scale(tanq_dm d, double factor) {
  return guarded([&] {
    check_dm(d);
    if (!std::isfinite(factor)) fail(TANQ_E_ARG, "scale factor must be finite");
    DeviceGuard g(d->device);
    launch_scale(d->ptr, d->n, d->prec, factor, d->stream);
  });
}

tanq_status tanq_mfma_rate(tanq_prec p, double* tflops) {
  return guarded([&] {
    check_prec(p);
    if (!tflops) fail(TANQ_E_ARG, "tflops is NULL");
    *tflops = mfma_rate_tflops(p);
  });
}

tanq_status tanq_dm_query(tanq_dm d, int* n, int* prec, uint64_t* elements, void** dev_ptr) {
  return guarded([&] {
    check_dm(d);
    if (n) *n = d->n;
    if (prec) *prec = (int)d->prec;
    if (elements) *elements = d->elements();
    if (dev_ptr) *dev_ptr = d->ptr;
  });
}

tanq_status tanq_dm_read(tanq_dm d, void* host, size_t bytes) {
  return guarded([&] {
    check_dm(d);
    if (!host) fail(TANQ_E_ARG, "host buffer is NULL");
    if (bytes != d->bytes()) fail(TANQ_E_ARG, "byte count must equal 4^n * element size");
    DeviceGuard g(d->device);
    TANQ_HIP(hipMemcpyAsync(host, d->ptr, bytes, hipMemcpyDeviceToHost, d->stream));
    TANQ_HIP(hipStreamSynchronize(d->stream));
  });
}

tanq_status tanq_dm_write(tanq_dm d, const void* host, size_t bytes) {
  return guarded([&] {
    check_dm(d);
    if (!host) fail(TANQ_E_ARG, "host buffer is NULL");
    if (bytes != d->bytes()) fail(TANQ_E_ARG, "byte count must equal 4^n * element size");
    DeviceGuard g(d->device);
    TANQ_HIP(hipMemcpyAsync(d->ptr, host, bytes, hipMemcpyHostToDevice, d->stream));
    TANQ_HIP(hipStreamSynchronize(d->stream));
  });
}

tanq_status tanq_dm_fill_random(tanq_dm d, uint64_t seed) {
  return guarded([&] {
    check_dm(d);
    if (seed >= (1ull << 23)) fail(TANQ_E_ARG, "seed must be below 2^23");
    DeviceGuard g(d->device);
    launch_fill_random(d->ptr, d->n, d->prec, seed, d->stream);
  });
}

tanq_status tanq_dm_gather(tanq_dm d, size_t count, const uint64_t* idx, void* host_out) {
  return guarded([&] {
    check_dm(d);
    if (count == 0) return;
    if (!idx || !host_out) fail(TANQ_E_ARG, "NULL argument");
    for (size_t i = 0; i < count; ++i)
      if (idx[i] >= d->elements()) fail(TANQ_E_ARG, "gather index out of range");
    DeviceGuard g(d->device);
    uint64_t* didx = nullptr;
    void* dout = nullptr;
    const size_t es = elem_size(d->prec);
    try {
      TANQ_HIP(hipMalloc((void**)&didx, count * sizeof(uint64_t)));
      TANQ_HIP(hipMalloc(&dout, count * es));
      TANQ_HIP(hipMemcpyAsync(didx, idx, count * sizeof(uint64_t), hipMemcpyHostToDevice, d->stream));
      launch_gather(d->ptr, d->prec, didx, count, dout, d->stream);
      TANQ_HIP(hipMemcpyAsync(host_out, dout, count * es, hipMemcpyDeviceToHost, d->stream));
      TANQ_HIP(hipStreamSynchronize(d->stream));
    } catch (...) {
      (void)hipStreamSynchronize(d->stream);
      dfree(didx);
      dfree(dout);
      throw;
    }
    dfree(didx);
    dfree(dout);
  });
}

tanq_status tanq_sync(tanq_dm d) {
  return guarded([&] {
    check_dm(d);
    DeviceGuard g(d->device);
    TANQ_HIP(hipStreamSynchronize(d->stream));
  });
}

// ---------------------------------------------------------------------------------------
// circuits
// ---------------------------------------------------------------------------------------

tanq_status tanq_circuit_create(int n, tanq_circuit* out) {
  return guarded([&] {
    if (!out) fail(TANQ_E_ARG, "out is NULL");
    if (n < 1 || n > MAX_N) fail(TANQ_E_ARG, "n must be in 1..17");
    tanq_circuit_s* c = new tanq_circuit_s;
    c->n = n;
    *out = c;
  });
}

tanq_status tanq_circuit_free(tanq_circuit c) {
  return guarded([&] { delete c; });
}

static void add_op(tanq_circuit c, int j, const int* qubits, int m, const double* K) {
  if (!c) fail(TANQ_E_ARG, "circuit handle is NULL");
  check_qubits(c->n, j, qubits, 3);
  if (m < 1) fail(TANQ_E_ARG, "at least one Kraus matrix is required");
  if (!K) fail(TANQ_E_ARG, "matrix pointer is NULL");
  HostOp op;
  op.j = j;
  op.m = m;
  for (int t = 0; t < j; ++t) op.q[t] = qubits[t];
  const size_t cnt = (size_t)m * (1u << j) * (1u << j) * 2;
  op.pool = std::make_shared<const std::vector<double>>(K, K + cnt);
  op.koff = 0;
  c->ops.push_back(std::move(op));
}

tanq_status tanq_circuit_add_gate(tanq_circuit c, int j, const int* qubits, const double* U) {
  return guarded([&] { add_op(c, j, qubits, 1, U); });
}

tanq_status tanq_circuit_add_kraus(tanq_circuit c, int j, const int* qubits, int m, const double* K) {
  return guarded([&] { add_op(c, j, qubits, m, K); });
}

tanq_status tanq_circuit_add_ops(tanq_circuit c, int count, const int* j, const int* qubits, const int* m,
                                 const int64_t* koff, const double* pool, size_t pool_doubles) {
  return guarded([&] {
    if (!c) fail(TANQ_E_ARG, "circuit handle is NULL");
    if (count < 0) fail(TANQ_E_ARG, "count must be >= 0");
    if (count == 0) return;
    if (!j || !qubits || !m || !koff || !pool) fail(TANQ_E_ARG, "NULL argument");
    auto shared = std::make_shared<const std::vector<double>>(pool, pool + pool_doubles);
    std::vector<HostOp> add((size_t)count);
    for (int i = 0; i < count; ++i) {
      check_qubits(c->n, j[i], qubits + 3 * i, 3);
      if (m[i] < 1) fail(TANQ_E_ARG, "at least one Kraus matrix is required");
      HostOp& op = add[i];
      op.j = j[i];
      op.m = m[i];
      for (int t = 0; t < op.j; ++t) op.q[t] = qubits[3 * i + t];
      if (koff[i] < 0 || (size_t)koff[i] + op.kdoubles() > pool_doubles)
        fail(TANQ_E_ARG, "operation " + std::to_string(i) + " reads past the matrix pool");
      op.pool = shared;
      op.koff = (size_t)koff[i];
    }
    c->ops.insert(c->ops.end(), std::make_move_iterator(add.begin()), std::make_move_iterator(add.end()));
  });
}

tanq_status tanq_circuit_size(tanq_circuit c, int* count) {
  return guarded([&] {
    if (!c || !count) fail(TANQ_E_ARG, "NULL argument");
    *count = (int)c->ops.size();
  });
}

// ---------------------------------------------------------------------------------------
// fusion
// ---------------------------------------------------------------------------------------

namespace {

// Measured milliseconds per apply, per (n, precision, k), filled by tanq_autotune or
// tanq_tuning_import; guarded by g_cost_mu.
double g_cost_ms[MAX_N + 1][2][4] = {};
std::mutex g_cost_mu;

double cost_get(int n, tanq_prec p, int k) {
  std::lock_guard<std::mutex> lk(g_cost_mu);
  return g_cost_ms[n][p == TANQ_F64 ? 0 : 1][k];
}

void cost_set(int n, tanq_prec p, int k, double ms) {
  std::lock_guard<std::mutex> lk(g_cost_mu);
  g_cost_ms[n][p == TANQ_F64 ? 0 : 1][k] = ms;
}

// Measured milliseconds per multi-superoperator pass of m 2-qubit superoperators, per (n,
// precision, m); guarded by g_cost_mu.
double g_pass_ms[MAX_N + 1][2][kPassMax + 1] = {};

double pass_cost_get(int n, tanq_prec p, int m) {
  std::lock_guard<std::mutex> lk(g_cost_mu);
  return g_pass_ms[n][p == TANQ_F64 ? 0 : 1][m];
}

void pass_cost_set(int n, tanq_prec p, int m, double ms) {
  std::lock_guard<std::mutex> lk(g_cost_mu);
  g_pass_ms[n][p == TANQ_F64 ? 0 : 1][m] = ms;
}

// Cost of one apply of width k, used to choose the fusion width when asked to: the
// autotuned time if there is one for (n, precision), else a model in units of one HBM
// pass over vec(rho) -- k <= 2 is bound by that pass, k = 3 by MFMA throughput (16 flop/B
// in FP64 and 32 flop/B in FP32 against machine balances of about 10 and 20 flop/B).
double apply_cost(int n, int k, tanq_prec p) {
  const double ms = cost_get(n, p, k);
  if (ms > 0.0) return ms;
  if (k <= 2) return 1.0;
  return 1.65;
}

// Cost of one pass of m 2-qubit superoperators: the measured time if there is one, else the
// 2-qubit apply cost scaled by a model of the pass (one HBM pass plus about a third of one
// per additional superoperator, as measured in FP64 at 16 qubits).
double pass_cost(int n, int m, tanq_prec p) {
  const double ms = pass_cost_get(n, p, m);
  if (ms > 0.0) return ms;
  return apply_cost(n, 2, p) * (1.0 + 0.35 * (m - 1));
}

// Cost of applying a planned block list the way tanq_apply_fused does (passes included).
double plan_cost(const std::vector<PlanBlock>& pl, int n, tanq_prec p) {
  auto at = [&](int j, const int** q) {
    *q = pl[j].qubits.data();
    return (int)pl[j].qubits.size();
  };
  const int lim = pass_limit();
  double c = 0.0;
  for (int i = 0; i < (int)pl.size();) {
    const int m = pass_run(at, i, (int)pl.size(), n, p, lim);
    c += m >= 2 ? pass_cost(n, m, p) : apply_cost(n, (int)pl[i].qubits.size(), p);
    i += m;
  }
  return c;
}

}  // namespace

tanq_status tanq_fuse(tanq_circuit c, int max_width, tanq_prec p, void* hip_stream, tanq_fused* out) {
  return guarded([&] {
    if (!c || !out) fail(TANQ_E_ARG, "NULL argument");
    *out = nullptr;
    check_prec(p);
    if (max_width < -2 || max_width > 3) fail(TANQ_E_ARG, "max_width must be -2..3");
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = c->n;
    const std::vector<PlanOp> pops = plan_ops(c->ops);
    int mode = max_width;
    std::vector<PlanBlock> plan;
    if (mode == TANQ_FUSE_AUTO) {
      double best = 1e300;
      for (int w = 2; w <= std::min(3, n); ++w) {
        std::vector<PlanBlock> pl = pass_order(plan_fusion(pops, n, w), n, p, pass_limit());
        const double cost = plan_cost(pl, n, p);
        if (cost < best) {
          best = cost;
          plan = std::move(pl);
          mode = w;
        }
      }
      if (n < 2) {
        plan = plan_fusion(pops, n, 1);
        mode = 1;
      }
    } else {
      plan = pass_order(plan_fusion(pops, n, mode), n, p, pass_limit());
    }

    std::unique_ptr<tanq_fused_s> f(new tanq_fused_s);
    f->n = n;
    f->prec = p;
    f->mode = mode;
    f->source_ops = (int)c->ops.size();
    TANQ_HIP(hipGetDevice(&f->device));
    const FuseLayout L = make_fuse_layout(c->ops, plan, p);
    f->blocks = L.host;
    for (int k = 0; k < 4; ++k) f->count_k[k] = L.count_k[k];

    if (!plan.empty()) {
      FuseOpDev* d_ops = nullptr;
      FuseBlockDev* d_blk = nullptr;
      double *d_kraus = nullptr, *d_sops = nullptr;
      auto cleanup = [&] {
        dfree(d_ops);
        dfree(d_blk);
        dfree(d_kraus);
        dfree(d_sops);
      };
      try {
        TANQ_HIP(hipMalloc((void**)&d_ops, L.ops.size() * sizeof(FuseOpDev)));
        TANQ_HIP(hipMalloc((void**)&d_blk, L.blocks.size() * sizeof(FuseBlockDev)));
        TANQ_HIP(hipMalloc((void**)&d_kraus, L.kraus.size() * sizeof(double)));
        TANQ_HIP(hipMalloc((void**)&d_sops, L.sop_elems * 2 * sizeof(double)));
        TANQ_HIP(hipMalloc((void**)&f->raw, L.raw_elems * 2 * sizeof(double)));
        TANQ_HIP(hipMalloc((void**)&f->packed, L.pack_bytes));
        TANQ_HIP(hipMemcpyAsync(d_ops, L.ops.data(), L.ops.size() * sizeof(FuseOpDev), hipMemcpyHostToDevice, s));
        TANQ_HIP(hipMemcpyAsync(d_blk, L.blocks.data(), L.blocks.size() * sizeof(FuseBlockDev), hipMemcpyHostToDevice, s));
        TANQ_HIP(hipMemcpyAsync(d_kraus, L.kraus.data(), L.kraus.size() * sizeof(double), hipMemcpyHostToDevice, s));
        run_fuse_kernels(L, d_ops, d_blk, d_kraus, d_sops, f->raw, f->packed, p, s);
        TANQ_HIP(hipStreamSynchronize(s));
      } catch (...) {
        (void)hipStreamSynchronize(s);
        cleanup();
        dfree(f->raw);
        dfree(f->packed);
        throw;
      }
      cleanup();
    }
    *out = f.release();
  });
}

tanq_status tanq_fuse_plan(tanq_circuit c, int max_width, int* op_block, int* nblocks) {
  return guarded([&] {
    if (!c || !nblocks) fail(TANQ_E_ARG, "NULL argument");
    if (max_width < -2 || max_width > 3 || max_width == 0) fail(TANQ_E_ARG, "max_width must be -2, -1, 1, 2 or 3");
    if (!c->ops.empty() && !op_block) fail(TANQ_E_ARG, "op_block is NULL");
    const std::vector<PlanBlock> plan = plan_fusion(plan_ops(c->ops), c->n, max_width);
    for (size_t b = 0; b < plan.size(); ++b)
      for (int oi : plan[b].ops) op_block[oi] = (int)b;
    *nblocks = (int)plan.size();
  });
}

tanq_status tanq_fuse_plan_ordered(tanq_circuit c, int max_width, tanq_prec p, int* op_block, int* nblocks) {
  return guarded([&] {
    if (!c || !nblocks) fail(TANQ_E_ARG, "NULL argument");
    if (max_width < -2 || max_width > 3 || max_width == 0) fail(TANQ_E_ARG, "max_width must be -2, -1, 1, 2 or 3");
    check_prec(p);
    if (!c->ops.empty() && !op_block) fail(TANQ_E_ARG, "op_block is NULL");
    const std::vector<PlanBlock> plan = pass_order(plan_fusion(plan_ops(c->ops), c->n, max_width), c->n, p, pass_limit());
    for (size_t b = 0; b < plan.size(); ++b)
      for (int oi : plan[b].ops) op_block[oi] = (int)b;
    *nblocks = (int)plan.size();
  });
}

tanq_status tanq_fused_info(tanq_fused f, tanq_fused_info_t* info) {
  return guarded([&] {
    if (!f || !info) fail(TANQ_E_ARG, "NULL argument");
    info->count = (int)f->blocks.size();
    for (int i = 0; i < 4; ++i) info->count_k[i] = f->count_k[i];
    info->source_ops = f->source_ops;
    info->max_width = f->mode;
    info->prec = (int)f->prec;
    info->n = f->n;
  });
}

tanq_status tanq_fused_free(tanq_fused f) {
  return guarded([&] {
    if (!f) return;
    (void)hipSetDevice(f->device);
    // applies of f may still be queued on any stream of the device
    (void)hipDeviceSynchronize();
    dfree(f->raw);
    dfree(f->packed);
    delete f;
  });
}

tanq_status tanq_fused_get(tanq_fused f, int idx, int* k, int* qubits, double* S) {
  return guarded([&] {
    if (!f) fail(TANQ_E_ARG, "fused handle is NULL");
    if (idx < 0 || idx >= (int)f->blocks.size()) fail(TANQ_E_ARG, "index out of range");
    const FusedBlockHost& b = f->blocks[idx];
    if (k) *k = b.k;
    if (qubits)
      for (int t = 0; t < b.k; ++t) qubits[t] = b.qubits[t];
    if (S) {
      DeviceGuard g(f->device);
      TANQ_HIP(hipMemcpy(S, f->raw + 2 * b.raw_off, ((size_t)1 << (4 * b.k)) * 2 * sizeof(double),
                         hipMemcpyDeviceToHost));
    }
  });
}

// ---------------------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------------------

tanq_status tanq_apply_superop(tanq_dm d, int k, const int* qubits, const double* S) {
  return guarded([&] {
    check_dm(d);
    check_qubits(d->n, k, qubits, 3);
    if (!S) fail(TANQ_E_ARG, "superoperator pointer is NULL");
    DeviceGuard g(d->device);
    const int slot = d->ring;
    d->ring = (d->ring + 1) % RING;
    TANQ_HIP(hipEventSynchronize(d->ev[slot]));  // previous upload from this slot is done
    const size_t cnt = ((size_t)1 << (4 * k)) * 2;
    double* host = d->pinned + slot * SLOT_DOUBLES;
    std::memcpy(host, S, cnt * sizeof(double));
    double* raw = d->s_raw_dev + slot * SLOT_DOUBLES;
    unsigned char* packed = d->s_packed_dev + slot * packed_bytes(3, TANQ_F64);
    TANQ_HIP(hipMemcpyAsync(raw, host, cnt * sizeof(double), hipMemcpyHostToDevice, d->stream));
    TANQ_HIP(hipEventRecord(d->ev[slot], d->stream));
    launch_pack_one(k, raw, packed, d->prec, d->stream);
    launch_apply(d->ptr, d->n, d->prec, k, qubits, packed, d->stream);
  });
}

tanq_status tanq_apply_fused_range(tanq_dm d, tanq_fused f, int begin, int end) {
  return guarded([&] {
    check_dm(d);
    if (!f) fail(TANQ_E_ARG, "fused handle is NULL");
    if (f->n != d->n) fail(TANQ_E_STATE, "fused list was built for a different qubit count");
    if (f->prec != d->prec) fail(TANQ_E_STATE, "fused list was packed for a different precision");
    if (begin < 0 || end > (int)f->blocks.size() || begin > end) fail(TANQ_E_ARG, "bad range");
    DeviceGuard g(d->device);
    const int lim = pass_limit();
    auto at = [&](int j, const int** q) {
      *q = f->blocks[j].qubits;
      return f->blocks[j].k;
    };
    for (int i = begin; i < end;) {
      const FusedBlockHost& b = f->blocks[i];
      const int m = pass_run(at, i, end, d->n, d->prec, lim);
      if (m >= 2) {
        const PassGeom* pg = nullptr;
        {
          std::lock_guard<std::mutex> lk(f->pass_mu);
          auto it = f->passes.find({i, m});
          if (it == f->passes.end()) {
            int q[2 * kPassMax];
            uint32_t off[kPassMax];
            const size_t es = d->prec == TANQ_F64 ? sizeof(double) : sizeof(float);
            for (int t = 0; t < m; ++t) {
              q[2 * t] = f->blocks[i + t].qubits[0];
              q[2 * t + 1] = f->blocks[i + t].qubits[1];
              off[t] = (uint32_t)((f->blocks[i + t].pack_off - b.pack_off) / es);
            }
            it = f->passes.emplace(std::make_pair(i, m), make_pass_geom(d->n, m, q, off, d->prec)).first;
          }
          pg = &it->second;  // map nodes are stable; entries are never erased
        }
        launch_pass(d->ptr, d->prec, *pg, f->packed + b.pack_off, d->stream);
        i += m;
      } else {
        launch_apply(d->ptr, d->n, d->prec, b.k, b.qubits, f->packed + b.pack_off, d->stream);
        ++i;
      }
    }
  });
}

tanq_status tanq_apply_fused(tanq_dm d, tanq_fused f) {
  if (!f) return set_error(TANQ_E_ARG, "fused handle is NULL");
  return tanq_apply_fused_range(d, f, 0, (int)f->blocks.size());
}

// ---------------------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------------------

tanq_status tanq_variant_count(int k, tanq_prec p, int* count) {
  return guarded([&] {
    if (!count) fail(TANQ_E_ARG, "count is NULL");
    check_prec(p);
    if (k == 1) {
      *count = 1;
      return;
    }
    if (k != 2 && k != 3) fail(TANQ_E_ARG, "k must be 1, 2 or 3");
    *count = variant_count(k, p);
  });
}

tanq_status tanq_variant_get(int k, tanq_prec p, int index, tanq_variant_t* out) {
  return guarded([&] {
    if (!out) fail(TANQ_E_ARG, "out is NULL");
    check_prec(p);
    if (k == 1) {
      if (index != 0) fail(TANQ_E_ARG, "k = 1 has one variant");
      *out = tanq_variant_t{1, (int)p, 0, 256, 0};
      return;
    }
    int tb = 0, th = 0, st = 0;
    if ((k != 2 && k != 3) || !variant_describe(k, p, index, &tb, &th, &st)) fail(TANQ_E_ARG, "no such variant");
    *out = tanq_variant_t{k, (int)p, tb, th, st};
  });
}

tanq_status tanq_variant_select(int k, tanq_prec p, int index) {
  return guarded([&] {
    check_prec(p);
    if (k == 1) {
      if (index != 0) fail(TANQ_E_ARG, "k = 1 has one variant");
      return;
    }
    if ((k != 2 && k != 3) || !variant_select(k, p, index)) fail(TANQ_E_ARG, "no such variant");
  });
}

tanq_status tanq_variant_selected(int k, tanq_prec p, int* index) {
  return guarded([&] {
    if (!index) fail(TANQ_E_ARG, "index is NULL");
    check_prec(p);
    if (k == 1) {
      *index = 0;
      return;
    }
    if (k != 2 && k != 3) fail(TANQ_E_ARG, "k must be 1, 2 or 3");
    *index = variant_selected(k, p);
  });
}

tanq_status tanq_variant_for(int n, int k, tanq_prec p, int* index) {
  return guarded([&] {
    if (!index) fail(TANQ_E_ARG, "index is NULL");
    check_prec(p);
    if (n < 1 || n > MAX_N) fail(TANQ_E_ARG, "n must be in 1..17");
    if (k == 1) {
      *index = 0;
      return;
    }
    if (k != 2 && k != 3) fail(TANQ_E_ARG, "k must be 1, 2 or 3");
    *index = variant_for(n, k, p);
  });
}

tanq_status tanq_tuning_export(char* buf, size_t cap, size_t* len) {
  return guarded([&] {
    if (!len) fail(TANQ_E_ARG, "len is NULL");
    std::string out;
    char line[160];
    for (int n = 1; n <= MAX_N; ++n)
      for (int pi = 0; pi < 2; ++pi) {
        const tanq_prec p = pi == 0 ? TANQ_F64 : TANQ_F32;
        for (int k = 1; k <= 3; ++k) {
          const double ms = cost_get(n, p, k);
          if (!(ms > 0.0)) continue;
          int tb = 0, th = 0, st = 0;
          if (k > 1) variant_describe(k, p, variant_for(n, k, p), &tb, &th, &st);
          std::snprintf(line, sizeof(line), "tune %d %d %s %d %d %d %.6g\n", n, k, pi == 0 ? "f64" : "f32", tb, th,
                        st, ms);
          out += line;
        }
        for (int m = 2; m <= kPassMax; ++m) {
          const double ms = pass_cost_get(n, p, m);
          if (!(ms > 0.0)) continue;
          std::snprintf(line, sizeof(line), "pass %d %s %d %.6g\n", n, pi == 0 ? "f64" : "f32", m, ms);
          out += line;
        }
      }
    *len = out.size() + 1;
    if (buf) {
      if (cap < out.size() + 1) fail(TANQ_E_ARG, "buffer too small");
      std::memcpy(buf, out.c_str(), out.size() + 1);
    }
  });
}

tanq_status tanq_tuning_import(const char* text) {
  return guarded([&] {
    if (!text) fail(TANQ_E_ARG, "text is NULL");
    struct Row {
      int n, k, variant;  // k = 0: a pass row, variant = superoperators per pass
      tanq_prec p;
      double ms;
    };
    std::vector<Row> rows;
    const char* cur = text;
    int lineno = 0;
    while (*cur) {
      const char* end = std::strchr(cur, '\n');
      std::string line = end ? std::string(cur, end) : std::string(cur);
      cur = end ? end + 1 : cur + line.size();
      ++lineno;
      if (line.empty() || line[0] == '#') continue;
      char prec[8] = {0};
      int n = 0, k = 0, tb = 0, th = 0, st = 0;
      double ms = 0.0;
      if (line.compare(0, 5, "pass ") == 0) {
        int m = 0;
        if (std::sscanf(line.c_str(), "pass %d %7s %d %lf", &n, prec, &m, &ms) != 4)
          fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + " is malformed");
        const std::string ps(prec);
        if (ps != "f64" && ps != "f32") fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + ": bad precision");
        const tanq_prec p = ps == "f64" ? TANQ_F64 : TANQ_F32;
        if (n < 1 || n > MAX_N || m < 2 || m > pass_max(p) || !(ms > 0.0))
          fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + ": out of range");
        rows.push_back({n, 0, m, p, ms});
        continue;
      }
      if (std::sscanf(line.c_str(), "tune %d %d %7s %d %d %d %lf", &n, &k, prec, &tb, &th, &st, &ms) != 7)
        fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + " is malformed");
      const std::string ps(prec);
      if (ps != "f64" && ps != "f32") fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + ": bad precision");
      const tanq_prec p = ps == "f64" ? TANQ_F64 : TANQ_F32;
      if (n < 1 || n > MAX_N || k < 1 || k > 3 || k > n || !(ms > 0.0))
        fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + ": out of range");
      int v = 0;
      if (k > 1) {
        v = variant_find(k, p, tb, th, st);
        if (v < 0) fail(TANQ_E_ARG, "tuning line " + std::to_string(lineno) + ": no such variant in this build");
      }
      rows.push_back({n, k, v, p, ms});
    }
    for (const Row& r : rows) {  // all lines valid: apply them
      if (r.k == 0) {
        pass_cost_set(r.n, r.p, r.variant, r.ms);
        continue;
      }
      if (r.k > 1) variant_tune(r.n, r.k, r.p, r.variant);
      cost_set(r.n, r.p, r.k, r.ms);
    }
  });
}

// A fixed pseudo-random 2^k x 2^k unitary (Gram-Schmidt on SplitMix64-seeded entries) and its
// superoperator conj(U) (x) U, local index row + 2^k col, row-major interleaved.
static std::vector<double> dense_unitary_superop(int k) {
  const int d = 1 << k, D = d * d;
  std::vector<std::complex<double>> U((size_t)d * d);
  uint64_t st = 0x5eed0000ull + (uint64_t)k;
  auto next = [&st]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 - 0.5;
  };
  for (auto& u : U) u = {next(), next()};
  for (int c = 0; c < d; ++c) {  // orthonormalise the columns
    for (int b = 0; b < c; ++b) {
      std::complex<double> dot = 0;
      for (int r = 0; r < d; ++r) dot += std::conj(U[(size_t)r * d + b]) * U[(size_t)r * d + c];
      for (int r = 0; r < d; ++r) U[(size_t)r * d + c] -= dot * U[(size_t)r * d + b];
    }
    double nrm = 0;
    for (int r = 0; r < d; ++r) nrm += std::norm(U[(size_t)r * d + c]);
    nrm = std::sqrt(nrm);
    for (int r = 0; r < d; ++r) U[(size_t)r * d + c] /= nrm;
  }
  std::vector<double> S((size_t)D * D * 2);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      // S[(r1 + d c1), (r2 + d c2)] = conj(U[c1][c2]) U[r1][r2]
      const int r1 = i % d, c1 = i / d, r2 = j % d, c2 = j / d;
      const std::complex<double> v = std::conj(U[(size_t)c1 * d + c2]) * U[(size_t)r1 * d + r2];
      S[2 * ((size_t)i * D + j)] = v.real();
      S[2 * ((size_t)i * D + j) + 1] = v.imag();
    }
  return S;
}

static void autotune_impl(tanq_dm d, int reps, bool dense, double* ms_per_apply) {
  check_dm(d);
  if (reps < 1) fail(TANQ_E_ARG, "reps must be >= 1");
  DeviceGuard g(d->device);
  const int n = d->n;
  const tanq_prec p = d->prec;
  if (dense) launch_fill_random(d->ptr, n, p, 1, d->stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TANQ_HIP(hipEventCreate(&e0));
  TANQ_HIP(hipEventCreate(&e1));
  double best_ms[4] = {0, 0, 0, 0};
  try {
      for (int k = 1; k <= std::min(3, n); ++k) {
        // identity (or dense unitary) superoperator, packed in slot 0 of the handle
        const int D = 1 << (2 * k);
        std::vector<double> S((size_t)D * D * 2, 0.0);
        if (dense)
          S = dense_unitary_superop(k);
        else
          for (int a = 0; a < D; ++a) S[2 * ((size_t)a * D + a)] = 1.0;
        double* raw = d->s_raw_dev;
        unsigned char* packed = d->s_packed_dev;
        TANQ_HIP(hipStreamSynchronize(d->stream));
        TANQ_HIP(hipMemcpy(raw, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
        launch_pack_one(k, raw, packed, p, d->stream);
        int lo[3], hi[3];
        for (int t = 0; t < k; ++t) {
          lo[t] = t;
          hi[t] = n - k + t;
        }
        const int nvar = (k == 1) ? 1 : variant_count(k, p);
        int best = (k == 1) ? 0 : variant_for(n, k, p);
        double best_t = 1e300;
        auto run = [&](int v, const int* q) {
          if (k == 1)
            launch_apply(d->ptr, n, p, k, q, packed, d->stream);
          else
            launch_apply_variant(d->ptr, n, p, k, v, q, packed, d->stream);
        };
        for (int v = 0; v < nvar; ++v) {
          run(v, lo);  // warm-up
          TANQ_HIP(hipEventRecord(e0, d->stream));
          for (int r = 0; r < reps; ++r) {
            run(v, lo);
            run(v, hi);
          }
          TANQ_HIP(hipEventRecord(e1, d->stream));
          TANQ_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          TANQ_HIP(hipEventElapsedTime(&ms, e0, e1));
          const double per = (double)ms / (2.0 * reps);
          if (per < best_t) {
            best_t = per;
            best = v;
          }
        }
        if (k > 1) variant_tune(n, k, p, best);
        best_ms[k] = best_t;
        cost_set(n, p, k, best_t);
      }
      // passes of m 2-qubit superoperators on the four highest qubits (whole 128-byte runs),
      // every superoperator the same identity (or dense unitary) operand
      if (2 * n - pass_tile_bits(p) >= kPassMinTileBits && pass_limit() >= 2) {
        const int D = 16;
        std::vector<double> S((size_t)D * D * 2, 0.0);
        if (dense)
          S = dense_unitary_superop(2);
        else
          for (int a = 0; a < D; ++a) S[2 * ((size_t)a * D + a)] = 1.0;
        TANQ_HIP(hipStreamSynchronize(d->stream));
        TANQ_HIP(hipMemcpy(d->s_raw_dev, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
        launch_pack_one(2, d->s_raw_dev, d->s_packed_dev, p, d->stream);
        const int a = n - 4, b = n - 3, c = n - 2, e = n - 1;
        const int cyc[6][2] = {{a, b}, {c, e}, {a, c}, {b, e}, {a, e}, {b, c}};
        const int mmax = std::min(pass_limit(), pass_max(p));
        for (int m = 2; m <= mmax; ++m) {
          int q[2 * kPassMax];
          uint32_t off[kPassMax] = {0};
          for (int t = 0; t < m; ++t) {
            q[2 * t] = cyc[t % 6][0];
            q[2 * t + 1] = cyc[t % 6][1];
          }
          const PassGeom pg = make_pass_geom(n, m, q, off, p);
          launch_pass(d->ptr, p, pg, d->s_packed_dev, d->stream);  // warm-up
          TANQ_HIP(hipEventRecord(e0, d->stream));
          for (int r = 0; r < 2 * reps; ++r) launch_pass(d->ptr, p, pg, d->s_packed_dev, d->stream);
          TANQ_HIP(hipEventRecord(e1, d->stream));
          TANQ_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          TANQ_HIP(hipEventElapsedTime(&ms, e0, e1));
          pass_cost_set(n, p, m, (double)ms / (2.0 * reps));
        }
      }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_per_apply)
    for (int k = 0; k < 4; ++k) ms_per_apply[k] = best_ms[k];
}

tanq_status tanq_set_pass_limit(int max_superops) {
  return guarded([&] { set_pass_limit(max_superops); });
}

tanq_status tanq_get_pass_limit(int* max_superops) {
  return guarded([&] {
    if (!max_superops) fail(TANQ_E_ARG, "max_superops is NULL");
    *max_superops = pass_limit();
  });
}

tanq_status tanq_fused_passes(tanq_fused f, int* passes, int* in_passes) {
  return guarded([&] {
    if (!f || !passes || !in_passes) fail(TANQ_E_ARG, "NULL argument");
    const int lim = pass_limit();
    auto at = [&](int j, const int** q) {
      *q = f->blocks[j].qubits;
      return f->blocks[j].k;
    };
    int np = 0, nin = 0;
    const int end = (int)f->blocks.size();
    for (int i = 0; i < end;) {
      const int m = pass_run(at, i, end, f->n, f->prec, lim);
      if (m >= 2) {
        ++np;
        nin += m;
      }
      i += m;
    }
    *passes = np;
    *in_passes = nin;
  });
}

tanq_status tanq_fused_launches(tanq_fused f, int* run_len, int cap, int* count) {
  return guarded([&] {
    if (!f || !count) fail(TANQ_E_ARG, "NULL argument");
    const int lim = pass_limit();
    auto at = [&](int j, const int** q) {
      *q = f->blocks[j].qubits;
      return f->blocks[j].k;
    };
    std::vector<int> runs;
    const int end = (int)f->blocks.size();
    for (int i = 0; i < end;) {
      const int m = pass_run(at, i, end, f->n, f->prec, lim);
      runs.push_back(m);
      i += m;
    }
    *count = (int)runs.size();
    if (run_len) {
      if (cap < (int)runs.size()) fail(TANQ_E_ARG, "run_len too small");
      std::copy(runs.begin(), runs.end(), run_len);
    }
  });
}

tanq_status tanq_pass_layout_info(int n, int m, const int* qubits, tanq_prec p, int* conflict_free,
                                  int* achievable) {
  return guarded([&] {
    if (!qubits || !conflict_free || !achievable) fail(TANQ_E_ARG, "NULL argument");
    check_prec(p);
    if (n < 1 || n > MAX_N) fail(TANQ_E_ARG, "n out of range");
    uint32_t off[kPassMax] = {0};
    int score = 0, bound = 0;
    (void)make_pass_geom(n, m, qubits, off, p, &score, &bound);
    *conflict_free = score;
    *achievable = bound;
  });
}

tanq_status tanq_autotune(tanq_dm d, int reps, double* ms_per_apply) {
  return guarded([&] { autotune_impl(d, reps, false, ms_per_apply); });
}

tanq_status tanq_autotune_dense(tanq_dm d, int reps, double* ms_per_apply) {
  return guarded([&] { autotune_impl(d, reps, true, ms_per_apply); });
}

// ---------------------------------------------------------------------------------------
// measurement statistics
// ---------------------------------------------------------------------------------------

tanq_status tanq_probs(tanq_dm d, double* host_out, int renormalize, double* trace_out) {
  return guarded([&] {
    check_dm(d);
    if (!host_out) fail(TANQ_E_ARG, "output buffer is NULL");
    DeviceGuard g(d->device);
    launch_diag(d->ptr, d->n, d->prec, d->probs_dev, d->partials, d->result_dev, renormalize, d->stream);
    TANQ_HIP(hipMemcpyAsync(host_out, d->probs_dev, (1ull << d->n) * sizeof(double), hipMemcpyDeviceToHost,
                            d->stream));
    double tr = 0.0;
    TANQ_HIP(hipMemcpyAsync(&tr, d->result_dev, sizeof(double), hipMemcpyDeviceToHost, d->stream));
    TANQ_HIP(hipStreamSynchronize(d->stream));
    if (trace_out) *trace_out = tr;
  });
}

static void check_readout(int n, const double* p01, const double* p10) {
  if ((p01 == nullptr) != (p10 == nullptr)) fail(TANQ_E_ARG, "give both readout arrays or neither");
  if (!p01) return;
  for (int t = 0; t < n; ++t)
    if (!(p01[t] >= 0.0 && p01[t] <= 1.0 && p10[t] >= 0.0 && p10[t] <= 1.0))
      fail(TANQ_E_ARG, "readout error probabilities must be in [0, 1]");
}

tanq_status tanq_probs_readout(tanq_dm d, const double* p01, const double* p10, double* host_out) {
  return guarded([&] {
    check_dm(d);
    if (!host_out || !p01 || !p10) fail(TANQ_E_ARG, "NULL argument");
    check_readout(d->n, p01, p10);
    DeviceGuard g(d->device);
    launch_diag(d->ptr, d->n, d->prec, d->probs_dev, d->partials, d->result_dev, 1, d->stream);
    launch_readout(d->probs_dev, d->n, p01, p10, d->stream);
    TANQ_HIP(hipMemcpyAsync(host_out, d->probs_dev, (1ull << d->n) * sizeof(double), hipMemcpyDeviceToHost,
                            d->stream));
    TANQ_HIP(hipStreamSynchronize(d->stream));
  });
}

}  // extern "C"

namespace tanq {

void sample_check(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10, uint64_t* host_out,
                  int* n, int* device) {
  check_dm(d);
  if (shots > 0 && !host_out) fail(TANQ_E_ARG, "NULL argument");
  if (seed >= (1ull << 23)) fail(TANQ_E_ARG, "seed must be below 2^23");
  if (shots > (1ull << 40)) fail(TANQ_E_ARG, "too many shots");
  check_readout(d->n, p01, p10);
  *n = d->n;
  *device = d->device;
}

void sample_run(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10, double* cdf_dev,
                uint64_t* out_dev, uint64_t* host_out) {
  DeviceGuard g(d->device);
  launch_diag(d->ptr, d->n, d->prec, d->probs_dev, d->partials, d->result_dev, 1, d->stream);
  if (p01) launch_readout(d->probs_dev, d->n, p01, p10, d->stream);
  launch_sample(d->probs_dev, d->n, cdf_dev, shots, seed, out_dev, d->stream);
  TANQ_HIP(hipMemcpyAsync(host_out, out_dev, shots * sizeof(uint64_t), hipMemcpyDeviceToHost, d->stream));
  TANQ_HIP(hipStreamSynchronize(d->stream));
}

}  // namespace tanq

extern "C" {

tanq_status tanq_sample(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10,
                        uint64_t* host_out) {
  return guarded([&] {
    int n = 0, device = 0;
    sample_check(d, shots, seed, p01, p10, host_out, &n, &device);
    if (shots == 0) return;
    DeviceGuard g(device);
    double* cdf = nullptr;
    uint64_t* out = nullptr;
    try {
      TANQ_HIP(hipMalloc((void**)&cdf, (1ull << n) * sizeof(double)));
      TANQ_HIP(hipMalloc((void**)&out, shots * sizeof(uint64_t)));
      sample_run(d, shots, seed, p01, p10, cdf, out, host_out);
    } catch (...) {
      (void)hipStreamSynchronize(d->stream);
      dfree(cdf);
      dfree(out);
      throw;
    }
    dfree(cdf);
    dfree(out);
  });
}

tanq_status tanq_dm_set_basis(tanq_dm d, uint64_t r, uint64_t c) {
  return guarded([&] {
    check_dm(d);
    const uint64_t dim = 1ull << d->n;
    if (r >= dim || c >= dim) fail(TANQ_E_ARG, "basis index out of range");
    DeviceGuard g(d->device);
    launch_init_basis(d->ptr, d->n, d->prec, r + (c << d->n), d->stream);
  });
}

tanq_status tanq_reduced_dm(tanq_dm d, int k, const int* keep, double* host_out) {
  return guarded([&] {
    check_dm(d);
    if (!host_out) fail(TANQ_E_ARG, "output is NULL");
    check_qubits(d->n, k, keep, 4);
    DeviceGuard g(d->device);
    int* kd = reinterpret_cast<int*>(d->masks_dev);  // small device scratch of the handle
    TANQ_HIP(hipMemcpyAsync(kd, keep, k * sizeof(int), hipMemcpyHostToDevice, d->stream));
    launch_reduced(d->ptr, d->n, d->prec, k, kd, d->result_dev, d->stream);
    TANQ_HIP(hipMemcpyAsync(host_out, d->result_dev, 2 * ((size_t)1 << (2 * k)) * sizeof(double),
                            hipMemcpyDeviceToHost, d->stream));
    TANQ_HIP(hipStreamSynchronize(d->stream));
  });
}

// chi_ij = Tr(B_ij^dag S) / 4 with B_ij = conj(sigma_j) (x) sigma_i, the orthogonal basis in which
// a one-qubit superoperator S = sum_ij chi_ij conj(sigma_j) (x) sigma_i (column stacking; sigma =
// I, X, Y, Z).  S is 4 x 4 complex, row-major, interleaved.
static void chi_from_superop(const double* S, double* chi) {
  static const double sig[4][2][2][2] = {
      {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}},
      {{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},
      {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},
      {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}},
  };
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double ar = 0.0, ai = 0.0;
      // B[(c1 r1)][(c2 r2)] = conj(sig_j[c1][c2]) * sig_i[r1][r2], row index r1 + 2 c1
      for (int c1 = 0; c1 < 2; ++c1)
        for (int r1 = 0; r1 < 2; ++r1)
          for (int c2 = 0; c2 < 2; ++c2)
            for (int r2 = 0; r2 < 2; ++r2) {
              const double xr = sig[j][c1][c2][0], xi = -sig[j][c1][c2][1];
              const double yr = sig[i][r1][r2][0], yi = sig[i][r1][r2][1];
              const double br = xr * yr - xi * yi, bi = xr * yi + xi * yr;
              const int row = r1 + 2 * c1, col = r2 + 2 * c2;
              const double sr = S[2 * (row * 4 + col)], si = S[2 * (row * 4 + col) + 1];
              // conj(B) * S
              ar += br * sr + bi * si;
              ai += br * si - bi * sr;
            }
      chi[2 * (i * 4 + j)] = ar / 4.0;
      chi[2 * (i * 4 + j) + 1] = ai / 4.0;
    }
}

tanq_status tanq_process_chi_1q(tanq_circuit c, int max_width, tanq_prec p, int in_qubit, int out_qubit,
                                double* chi_out, double* superop_out) {
  return guarded([&] {
    if (!c || !chi_out) fail(TANQ_E_ARG, "NULL argument");
    if (in_qubit < 0 || in_qubit >= c->n || out_qubit < 0 || out_qubit >= c->n)
      fail(TANQ_E_ARG, "qubit out of range");
    tanq_fused f = nullptr;
    tanq_dm d = nullptr;
    auto cleanup = [&] {
      if (d) tanq_dm_free(d);
      if (f) tanq_fused_free(f);
    };
    try {
      if (tanq_fuse(c, max_width, p, nullptr, &f) != TANQ_OK) fail(TANQ_E_STATE, tanq_last_error());
      if (tanq_dm_init(c->n, p, nullptr, &d) != TANQ_OK) fail(TANQ_E_STATE, tanq_last_error());
      double S[32];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          // input |a><b| on in_qubit, |0><0| elsewhere; output reduced to out_qubit
          if (tanq_dm_set_basis(d, (uint64_t)a << in_qubit, (uint64_t)b << in_qubit) != TANQ_OK ||
              tanq_apply_fused(d, f) != TANQ_OK)
            fail(TANQ_E_STATE, tanq_last_error());
          double red[8];
          if (tanq_reduced_dm(d, 1, &out_qubit, red) != TANQ_OK) fail(TANQ_E_STATE, tanq_last_error());
          // column a + 2b of S is vec(E(|a><b|)) = (red[0][0], red[1][0], red[0][1], red[1][1])
          const int col = a + 2 * b;
          for (int rr = 0; rr < 2; ++rr)
            for (int cc = 0; cc < 2; ++cc) {
              const int row = rr + 2 * cc;
              S[2 * (row * 4 + col)] = red[2 * (rr * 2 + cc)];
              S[2 * (row * 4 + col) + 1] = red[2 * (rr * 2 + cc) + 1];
            }
        }
      chi_from_superop(S, chi_out);
      if (superop_out) std::memcpy(superop_out, S, sizeof(S));
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  });
}

tanq_status tanq_expect_pauli_batch(tanq_dm d, int count, const char* const* paulis, double* out_re,
                                    double* out_im) {
  return guarded([&] {
    check_dm(d);
    if (count < 0 || (count > 0 && (!paulis || !out_re))) fail(TANQ_E_ARG, "NULL argument");
    DeviceGuard g(d->device);
    constexpr int CHUNK = 1024;
    std::vector<uint64_t> masks(3 * CHUNK);
    std::vector<double> res(2 * CHUNK);
    for (int base = 0; base < count; base += CHUNK) {
      const int cnt = std::min(CHUNK, count - base);
      for (int i = 0; i < cnt; ++i) parse_pauli(d->n, paulis[base + i], &masks[3 * i]);
      TANQ_HIP(hipMemcpyAsync(d->masks_dev, masks.data(), 3 * cnt * sizeof(uint64_t), hipMemcpyHostToDevice,
                              d->stream));
      launch_pauli(d->ptr, d->n, d->prec, cnt, d->masks_dev, d->partials, d->result_dev, d->stream);
      TANQ_HIP(hipMemcpyAsync(res.data(), d->result_dev, 2 * cnt * sizeof(double), hipMemcpyDeviceToHost,
                              d->stream));
      TANQ_HIP(hipStreamSynchronize(d->stream));
      for (int i = 0; i < cnt; ++i) {
        out_re[base + i] = res[2 * i];
        if (out_im) out_im[base + i] = res[2 * i + 1];
      }
    }
  });
}

tanq_status tanq_dm_compare(tanq_dm a, tanq_dm b, double* out3) {
  return guarded([&] {
    check_dm(a);
    check_dm(b);
    if (!out3) fail(TANQ_E_ARG, "out3 is NULL");
    if (a->n != b->n) fail(TANQ_E_ARG, "different qubit counts");
    if (a->device != b->device) fail(TANQ_E_ARG, "handles live on different devices");
    DeviceGuard g(a->device);
    TANQ_HIP(hipStreamSynchronize(b->stream));
    launch_compare(a->ptr, a->prec, b->ptr, b->prec, a->elements(), a->partials, a->result_dev, a->stream);
    TANQ_HIP(hipMemcpyAsync(out3, a->result_dev, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
    TANQ_HIP(hipStreamSynchronize(a->stream));
  });
}

tanq_status tanq_expect_pauli_c(tanq_dm d, const char* pauli, double* re, double* im) {
  const char* arr[1] = {pauli};
  double r = 0.0, i = 0.0;
  tanq_status st = tanq_expect_pauli_batch(d, 1, arr, &r, &i);
  if (st == TANQ_OK) {
    if (re) *re = r;
    if (im) *im = i;
  }
  return st;
}

tanq_status tanq_expect_pauli(tanq_dm d, const char* pauli, double* out) {
  if (!out) return set_error(TANQ_E_ARG, "out is NULL");
  return tanq_expect_pauli_c(d, pauli, out, nullptr);
}

}  // extern "C"
