// Continuous-batching server for many small noisy circuits (density matrices of uneven size).
//
// Requests are admitted by device-memory footprint and slot count; each admitted request's
// state vec(rho) stays resident in a device arena until its results are read back.  A
// scheduler thread owns one HIP stream.  Each iteration it
//   1. admits waiting requests (FIFO) while their footprint fits: fuses the circuit on the GPU
//      (superoperators, FP64 composition, packing, all blocks widened to the server's width)
//      and initialises rho = |0..0><0..0|;
//   2. builds the work of S steps: in step s every active request contributes its next fused
//      superoperator as one batch item, split into chunks of tiles;
//   3. launches the S batched kernels (captured once in a hipGraph per work buffer and
//      replayed), each applying one superoperator to every active state at once;
//   4. for requests whose last superoperator ran, reduces probabilities and Pauli expectations
//      in FP64 and copies them to pinned host memory; completion is observed with events.
// Requests that arrive while others are on the GPU join at the next iteration, so their work
// overlaps with the requests already resident.  A request's arithmetic does not depend on the
// other requests in a launch (fixed tile shape per size, no cross-request reduction), so its
// result is the same alone and in the mix.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "abi_util.hpp"
#include "circuit.hpp"

namespace tanq {

// First-fit sub-allocator over one region (offsets in bytes, 256-byte granules).
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(size_t size, size_t* off) {
    size = align256(size == 0 ? 1 : size);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= size) {
        *off = it->first;
        const size_t rest = it->second - size, start = it->first + size;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += size;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t size) {
    size = align256(size == 0 ? 1 : size);
    used_ -= size;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + size == next->first) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += size;
        return;
      }
    }
    free_[off] = size;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct ServeRequest {
  uint64_t ticket = 0;
  int n = 0;
  std::vector<HostOp> ops;
  bool want_probs = false;
  std::vector<std::array<uint64_t, 3>> paulis;
  int state = 0;  // 0 pending, 1 admitted (in flight), 2 done
  tanq_status status = TANQ_OK;
  std::string error;
  int slot = -1;
  // device arena regions
  size_t keep_off = 0, keep_size = 0;  // rho + packed operands, held until completion
  // pinned result region
  size_t res_off = 0, res_size = 0;
  size_t rho_off = 0;
  std::vector<size_t> pack_off;  // per fused block (absolute arena offsets)
  std::vector<ApplyGeom> geom;   // per fused block
  size_t cursor = 0;
  bool finishing = false;  // its reductions are queued; leaves the resident set
  tanq_status drop = TANQ_OK;  // TANQ_E_CANCELED / TANQ_E_TIMEOUT: stop and free it, no outputs
  bool outputs_queued = false; // its reductions were queued (a later cancel no longer applies)
  // admission work (uploads, superoperators, composition, packing, state initialisation) runs
  // on the admission stream; the request joins the batched steps once this event completed
  hipEvent_t ready_ev = nullptr;
  bool ready = false;
  double deadline = 0;         // server clock time after which it times out (0: none)
  FuseLayout layout;  // planned at submit (exact footprint); consumed at admission
  // results
  double trace = 0.0;
  std::vector<double> probs, pauli;
  double t_submit = 0, t_admit = 0, t_done = 0;
  size_t footprint = 0;
};

constexpr int kServeMaxN = 14;
// Chunk-list capacity per slot and step.  The whole work list (every step's items and chunk
// capacity) is copied to the device before each iteration's launches, so its size is on the
// serving path: 64 per slot (4096 chunks per step at 64 slots, 0.7 MiB per 8-step iteration)
// rather than 256 (2.2 MiB); the chunker makes chunks coarser when a step would exceed it.
constexpr uint64_t kChunksPerItem = 64;
constexpr uint64_t kMinChunkTiles = 4;    // smallest chunk (guided sizes shrink towards it)

static size_t state_bytes(int n, tanq_prec p) { return ((size_t)1 << (2 * n)) * elem_size(p); }

// Device bytes a request holds while its fusion runs: rho and the packed operands (kept to the
// end) plus the fusion tables, superoperators and FP64 compositions (released after fusion).
static size_t request_footprint(int n, tanq_prec p, const FuseLayout& L) {
  return align256(state_bytes(n, p)) + L.pack_bytes + align256(L.ops.size() * sizeof(FuseOpDev)) +
         align256(L.blocks.size() * sizeof(FuseBlockDev)) + align256(L.kraus.size() * sizeof(double)) +
         align256(L.sop_elems * 2 * sizeof(double)) + align256(L.raw_elems * 2 * sizeof(double)) + 7 * 256;
}

}  // namespace tanq

using namespace tanq;

struct tanq_server_s {
  tanq_server_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;      // batched launches, reductions, result copies
  hipStream_t adm_stream = nullptr;  // admission: fusion kernels and state initialisation
  std::chrono::steady_clock::time_point t0;

  // device and pinned memory
  unsigned char* arena_base = nullptr;
  Arena arena;
  unsigned char* pinned_base = nullptr;
  Arena pinned;
  // shared reduction scratch (stream-ordered)
  double* probs_dev = nullptr;
  double* partials = nullptr;
  double* result_dev = nullptr;
  uint64_t* masks_dev = nullptr;

  // step work buffers (double-buffered), pinned and device, with one graph each
  size_t items_per_step = 0, chunks_per_step = 0, work_bytes = 0;
  uint64_t grid = 1;  // workgroups of the batched kernel's persistent grid
  unsigned char* work_host[2] = {nullptr, nullptr};
  unsigned char* work_dev[2] = {nullptr, nullptr};
  hipEvent_t work_ev[2] = {nullptr, nullptr};
  bool work_ev_used[2] = {false, false};
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int flip = 0;

  // fusion staging: pinned regions released when their event completes
  struct Staged {
    hipEvent_t ev;
    size_t off, size;
  };
  std::deque<Staged> staged;
  std::vector<hipEvent_t> event_pool;

  // completion tracking
  struct Finishing {
    hipEvent_t ev;
    std::vector<ServeRequest*> reqs;
  };
  std::deque<Finishing> finishing;

  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<ServeRequest*> pending;
  std::vector<ServeRequest*> active;
  size_t rr_next = 0;  // cohort scheduling: where the next cohort starts in `active`
  std::unordered_map<uint64_t, std::unique_ptr<ServeRequest>> all;
  std::vector<int> free_slots;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool failed = false;
  std::string fail_msg;
  std::thread worker;

  // statistics (written by the scheduler, read by tanq_server_stats_get)
  std::atomic<uint64_t> n_submitted{0}, n_admitted{0}, n_completed{0}, n_rejected{0}, n_launches{0}, n_steps{0};
  std::atomic<uint64_t> n_tiles{0}, n_chunks{0}, n_dropped{0};
  std::atomic<size_t> bytes_in_use{0}, peak_bytes{0};
  std::atomic<int> n_active{0};

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    TANQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }
  void put_event(hipEvent_t e) { event_pool.push_back(e); }

  // Work buffer layout per step s: [chunk count u32, next-chunk counter u32 (padded to 256)]
  // [items] [chunks]
  size_t step_bytes() const {
    return 256 + align256(items_per_step * sizeof(BatchItem)) + align256(chunks_per_step * sizeof(BatchChunk));
  }
  uint32_t* step_count(unsigned char* base, int s) const { return (uint32_t*)(base + s * step_bytes()); }
  BatchItem* step_items(unsigned char* base, int s) const { return (BatchItem*)(base + s * step_bytes() + 256); }
  BatchChunk* step_chunks(unsigned char* base, int s) const {
    return (BatchChunk*)(base + s * step_bytes() + 256 + align256(items_per_step * sizeof(BatchItem)));
  }

  void record_launches(int b);
  void admit_one(ServeRequest* r);
  void run_iteration();
  void finalize_done(bool block);
  void loop();
};

// --------------------------------------------------------------------------------------
// scheduler
// --------------------------------------------------------------------------------------

void tanq_server_s::record_launches(int b) {
  // the S batched launches of one iteration, reading work buffer b
  const int S = cfg.steps_per_launch;
  TANQ_HIP(hipMemcpyAsync(work_dev[b], work_host[b], work_bytes, hipMemcpyHostToDevice, stream));
  for (int s = 0; s < S; ++s)
    launch_batch(cfg.width, (tanq_prec)cfg.prec, step_items(work_dev[b], s), step_chunks(work_dev[b], s),
                 step_count(work_dev[b], s), stream);
}

void tanq_server_s::admit_one(ServeRequest* r) {
  const tanq_prec p = (tanq_prec)cfg.prec;
  const int w = cfg.width;
  const FuseLayout& L = r->layout;

  // persistent region: rho followed by the packed operands
  const size_t rho_b = align256(state_bytes(r->n, p));
  r->keep_size = rho_b + L.pack_bytes;
  // temporary region: tables, Kraus pool, superoperators, FP64 compositions
  const size_t ops_b = align256(L.ops.size() * sizeof(FuseOpDev));
  const size_t blk_b = align256(L.blocks.size() * sizeof(FuseBlockDev));
  const size_t kr_b = align256(L.kraus.size() * sizeof(double));
  const size_t sop_b = align256(L.sop_elems * 2 * sizeof(double));
  const size_t raw_b = align256(L.raw_elems * 2 * sizeof(double));
  const size_t tmp_size = ops_b + blk_b + kr_b + sop_b + raw_b;
  size_t keep_off = 0, tmp_off = 0, stage_off = 0;
  if (!arena.alloc(r->keep_size, &keep_off)) fail(TANQ_E_OOM, "arena exhausted at admission");
  if (!arena.alloc(tmp_size, &tmp_off)) {
    arena.release(keep_off, r->keep_size);
    fail(TANQ_E_OOM, "arena exhausted at admission");
  }
  const size_t stage_size = ops_b + blk_b + kr_b;
  if (!pinned.alloc(stage_size, &stage_off)) {
    arena.release(keep_off, r->keep_size);
    arena.release(tmp_off, tmp_size);
    fail(TANQ_E_OOM, "pinned staging exhausted at admission");
  }
  r->keep_off = keep_off;
  r->rho_off = keep_off;
  unsigned char* tmp = arena_base + tmp_off;
  unsigned char* stg = pinned_base + stage_off;
  std::memcpy(stg, L.ops.data(), L.ops.size() * sizeof(FuseOpDev));
  std::memcpy(stg + ops_b, L.blocks.data(), L.blocks.size() * sizeof(FuseBlockDev));
  std::memcpy(stg + ops_b + blk_b, L.kraus.data(), L.kraus.size() * sizeof(double));
  TANQ_HIP(hipMemcpyAsync(tmp, stg, stage_size, hipMemcpyHostToDevice, adm_stream));
  hipEvent_t ev = get_event();
  TANQ_HIP(hipEventRecord(ev, adm_stream));
  staged.push_back({ev, stage_off, stage_size});
  run_fuse_kernels(L, (const FuseOpDev*)tmp, (const FuseBlockDev*)(tmp + ops_b), (const double*)(tmp + ops_b + blk_b),
                   (double*)(tmp + ops_b + blk_b + kr_b), (double*)(tmp + ops_b + blk_b + kr_b + sop_b),
                   arena_base + keep_off + rho_b, p, adm_stream);
  // every later user of this region is ordered after the fusion kernels: other admissions run
  // on the same stream, and only admissions allocate from the arena
  arena.release(tmp_off, tmp_size);
  launch_init_zero(arena_base + r->rho_off, r->n, p, adm_stream);
  // the batched launches (on the other stream) take the request only once this has completed,
  // checked on the host, so they never wait on the admission stream
  r->ready_ev = get_event();
  TANQ_HIP(hipEventRecord(r->ready_ev, adm_stream));
  r->ready = false;

  r->pack_off.resize(L.host.size());
  r->geom.resize(L.host.size());
  const int vb = batch_tile_bits(w, p);
  for (size_t i = 0; i < L.host.size(); ++i) {
    r->pack_off[i] = keep_off + rho_b + L.host[i].pack_off;
    r->geom[i] = make_apply_geom(r->n, w, L.host[i].qubits, vb, p);
  }
  r->cursor = 0;
  r->t_admit = now();
  r->layout = FuseLayout();  // host tables no longer needed
}

void tanq_server_s::run_iteration() {
  const int S = cfg.steps_per_launch;
  const int b = flip;
  flip ^= 1;
  if (work_ev_used[b]) TANQ_HIP(hipEventSynchronize(work_ev[b]));  // buffer b's last copy is done
  unsigned char* W = work_host[b];
  std::vector<ServeRequest*> done_now;
  // the requests this iteration advances: all of them, or a round-robin cohort whose states
  // total at most cohort_bytes
  std::vector<ServeRequest*> cohort;
  if (cfg.cohort_bytes == 0 || active.size() <= 1) {
    cohort = active;
  } else {
    const tanq_prec p = (tanq_prec)cfg.prec;
    if (rr_next >= active.size()) rr_next = 0;
    size_t bytes = 0;
    for (size_t i = 0; i < active.size(); ++i) {
      ServeRequest* r = active[(rr_next + i) % active.size()];
      const size_t sb = state_bytes(r->n, p);
      if (!cohort.empty() && bytes + sb > cfg.cohort_bytes) break;
      cohort.push_back(r);
      bytes += sb;
    }
    rr_next = (rr_next + cohort.size()) % active.size();
  }
  // requests whose admission work has not completed yet sit this iteration out (and cannot be
  // dropped or finished yet: their memory is still being written on the admission stream)
  for (ServeRequest* r : active)
    if (!r->ready) {
      const hipError_t q = hipEventQuery(r->ready_ev);
      if (q == hipErrorNotReady) continue;
      TANQ_HIP(q);
      put_event(r->ready_ev);
      r->ready_ev = nullptr;
      r->ready = true;
    }
  cohort.erase(std::remove_if(cohort.begin(), cohort.end(), [](ServeRequest* r) { return !r->ready; }),
               cohort.end());
  // dropped requests (cancelled or timed out) leave now: no further applies, no outputs; the
  // event recorded after this iteration's launches orders the release of their memory after
  // every launch already queued for them
  {
    std::lock_guard<std::mutex> lk(mu);
    const double t = now();
    for (ServeRequest* r : active)
      if (!r->finishing && r->drop == TANQ_OK && r->deadline > 0 && t > r->deadline) r->drop = TANQ_E_TIMEOUT;
    for (ServeRequest* r : active)
      if (r->ready && !r->finishing && r->drop != TANQ_OK) {
        r->finishing = true;
        done_now.push_back(r);
      }
  }
  cohort.erase(std::remove_if(cohort.begin(), cohort.end(), [](ServeRequest* r) { return r->finishing; }),
               cohort.end());
  // a circuit with no operations has nothing to apply: its outputs are those of |0..0><0..0|
  for (ServeRequest* r : cohort)
    if (r->geom.empty() && !r->finishing) {
      r->finishing = true;
      done_now.push_back(r);
    }
  bool any_item = false;  // some step has work (otherwise the launches are skipped)
  for (int s = 0; s < S; ++s) {
    uint32_t ni = 0, nc = 0;
    BatchItem* items = step_items(W, s);
    BatchChunk* chunks = step_chunks(W, s);
    for (ServeRequest* r : cohort) {
      if (r->cursor >= r->geom.size()) continue;
      BatchItem& it = items[ni];
      it.rho = (uint64_t)(uintptr_t)(arena_base + r->rho_off);
      it.frag = (uint64_t)(uintptr_t)(arena_base + r->pack_off[r->cursor]);
      it.g = r->geom[r->cursor];
      ++ni;
      r->cursor += 1;
      if (r->cursor == r->geom.size()) {
        r->finishing = true;
        done_now.push_back(r);
      }
    }
    // Chunks, claimed in list order by the persistent grid: items by decreasing size, cut with
    // guided sizes (remaining tiles of the step / grid size, at least kMinChunkTiles), so the
    // first claims are long and the last ones short and the workgroups finish close together.
    // An item boundary may cut a chunk short; a chunk never spans two items.
    std::vector<uint32_t> order(ni);
    std::vector<uint64_t> ntiles(ni);
    uint64_t remaining = 0;
    for (uint32_t i = 0; i < ni; ++i) {
      order[i] = i;
      ntiles[i] = items[i].g.ntiles;
      remaining += ntiles[i];
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return ntiles[a] > ntiles[b]; });
    for (uint32_t oi = 0; oi < ni; ++oi) {
      const uint32_t i = order[oi];
      const uint64_t nt = ntiles[i];
      for (uint64_t t0 = 0; t0 < nt;) {
        // keep room for one chunk per item still to come, whatever the sizes
        const uint64_t later = ni - 1 - oi;
        if ((uint64_t)nc + later >= chunks_per_step) fail(TANQ_E_STATE, "chunk list overflow");
        const uint64_t room = chunks_per_step - nc - later;
        uint64_t ct = std::max<uint64_t>(kMinChunkTiles, (remaining + grid - 1) / grid);
        ct = std::max<uint64_t>(ct, (remaining + room - 1) / room);
        ct = std::min<uint64_t>(ct, nt - t0);
        chunks[nc].item = i;
        chunks[nc].tile_begin = (uint32_t)t0;
        chunks[nc].tile_end = (uint32_t)(t0 + ct);
        chunks[nc].pad = 0;
        ++nc;
        t0 += ct;
        remaining -= ct;
      }
    }
    step_count(W, s)[0] = nc;
    step_count(W, s)[1] = 0;  // next unclaimed chunk, reset by the copy before each launch
    any_item = any_item || ni > 0;
    for (uint32_t i = 0; i < ni; ++i) n_tiles += ntiles[i];
    n_chunks += nc;
    if (nc) ++n_steps;
  }
  if (any_item) {
    if (graph[b]) {
      TANQ_HIP(hipGraphLaunch(graph[b], stream));
    } else {
      record_launches(b);
    }
    n_launches += 1;
    TANQ_HIP(hipEventRecord(work_ev[b], stream));
    work_ev_used[b] = true;
  } else if (done_now.empty()) {
    // every resident request is still being admitted: wait for the oldest instead of spinning
    for (ServeRequest* r : active)
      if (!r->ready) {
        TANQ_HIP(hipEventSynchronize(r->ready_ev));
        break;
      }
  }

  if (!done_now.empty()) {
    const tanq_prec p = (tanq_prec)cfg.prec;
    for (ServeRequest* r : done_now) {
      {
        std::lock_guard<std::mutex> lk(mu);
        if (r->drop != TANQ_OK) continue;  // no outputs
        r->outputs_queued = true;
      }
      unsigned char* rho = arena_base + r->rho_off;
      double* hres = (double*)(pinned_base + r->res_off);
      launch_diag(rho, r->n, p, probs_dev, partials, result_dev, 1, stream);
      TANQ_HIP(hipMemcpyAsync(hres, result_dev, sizeof(double), hipMemcpyDeviceToHost, stream));
      if (r->want_probs)
        TANQ_HIP(hipMemcpyAsync(hres + 1, probs_dev, ((size_t)1 << r->n) * sizeof(double), hipMemcpyDeviceToHost,
                                stream));
      if (!r->paulis.empty()) {
        const int cnt = (int)r->paulis.size();
        TANQ_HIP(hipMemcpyAsync(masks_dev, r->paulis.data(), 3 * cnt * sizeof(uint64_t), hipMemcpyHostToDevice,
                                stream));
        launch_pauli(rho, r->n, p, cnt, masks_dev, partials, result_dev, stream);
        const size_t off = 1 + (r->want_probs ? ((size_t)1 << r->n) : 0);
        TANQ_HIP(hipMemcpyAsync(hres + off, result_dev, 2 * cnt * sizeof(double), hipMemcpyDeviceToHost, stream));
      }
    }
    hipEvent_t ev = get_event();
    TANQ_HIP(hipEventRecord(ev, stream));
    finishing.push_back({ev, done_now});
    active.erase(std::remove_if(active.begin(), active.end(), [](ServeRequest* r) { return r->finishing; }),
                 active.end());
  }
}

void tanq_server_s::finalize_done(bool block) {
  // staging regions whose uploads finished
  while (!staged.empty()) {
    hipError_t q = hipEventQuery(staged.front().ev);
    if (q == hipErrorNotReady) break;
    TANQ_HIP(q);
    pinned.release(staged.front().off, staged.front().size);
    put_event(staged.front().ev);
    staged.pop_front();
  }
  while (!finishing.empty()) {
    Finishing& f = finishing.front();
    if (block) {
      TANQ_HIP(hipEventSynchronize(f.ev));
    } else {
      hipError_t q = hipEventQuery(f.ev);
      if (q == hipErrorNotReady) break;
      TANQ_HIP(q);
    }
    const double t = now();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (ServeRequest* r : f.reqs) {
        if (!r->outputs_queued) {
          r->status = r->drop;
          r->error = r->drop == TANQ_E_CANCELED ? "request cancelled" : "request timed out";
        } else {
          const double* hres = (const double*)(pinned_base + r->res_off);
          r->trace = hres[0];
          size_t off = 1;
          if (r->want_probs) {
            r->probs.assign(hres + 1, hres + 1 + ((size_t)1 << r->n));
            off += (size_t)1 << r->n;
          }
          r->pauli.resize(r->paulis.size());
          for (size_t i = 0; i < r->paulis.size(); ++i) r->pauli[i] = hres[off + 2 * i];
        }
        arena.release(r->keep_off, r->keep_size);
        pinned.release(r->res_off, r->res_size);
        free_slots.push_back(r->slot);
        r->slot = -1;
        r->t_done = t;
        r->state = 2;
        if (!r->outputs_queued)
          ++n_dropped;
        else
          ++n_completed;
      }
    }
    put_event(f.ev);
    finishing.pop_front();
    cv_done.notify_all();
  }
}

void tanq_server_s::loop() {
  try {
    TANQ_HIP(hipSetDevice(device));
    for (;;) {
      std::vector<ServeRequest*> to_admit;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (pending.empty() && active.empty() && finishing.empty() && staged.empty()) {
          if (stop) break;
          cv_submit.wait_for(lk, std::chrono::microseconds(500));
          continue;
        }
        // queued requests past their deadline leave the queue
        if (cfg.request_timeout_s > 0 && !pending.empty()) {
          const double t = now();
          bool any = false;
          for (auto it = pending.begin(); it != pending.end();) {
            ServeRequest* r = *it;
            if (r->deadline > 0 && t > r->deadline) {
              r->status = TANQ_E_TIMEOUT;
              r->error = "request timed out";
              r->t_done = t;
              r->state = 2;
              ++n_dropped;
              it = pending.erase(it);
              any = true;
            } else {
              ++it;
            }
          }
          if (any) cv_done.notify_all();
        }
        // FIFO admission by slot and footprint (head-of-line: a request that does not fit
        // waits for memory instead of being overtaken)
        while (!pending.empty() && !free_slots.empty()) {
          ServeRequest* r = pending.front();
          if (arena.used() + r->footprint > arena.size()) break;
          pending.pop_front();
          r->slot = free_slots.back();
          free_slots.pop_back();
          r->state = 1;
          to_admit.push_back(r);
        }
      }
      bool deferred = false;  // a request went back to the queue for lack of memory
      for (ServeRequest* r : to_admit) {
        size_t roff = 0;
        r->res_size = (1 + (r->want_probs ? ((size_t)1 << r->n) : 0) + 2 * r->paulis.size()) * sizeof(double);
        bool ok = pinned.alloc(r->res_size, &roff);
        r->res_off = roff;
        try {
          if (!ok) fail(TANQ_E_OOM, "pinned result space exhausted");
          admit_one(r);
          active.push_back(r);
          ++n_admitted;
        } catch (const Error& e) {
          if (ok) pinned.release(roff, r->res_size);
          std::lock_guard<std::mutex> lk(mu);
          if (e.code == TANQ_E_OOM) {
            // arena fragmentation or result space held by unreleased results: retry later
            deferred = true;
            r->state = 0;
            free_slots.push_back(r->slot);
            r->slot = -1;
            pending.push_front(r);
          } else {
            r->status = e.code;
            r->error = e.what();
            r->state = 2;
            free_slots.push_back(r->slot);
            r->slot = -1;
            cv_done.notify_all();
          }
        }
      }
      if (!active.empty()) {
        run_iteration();
      } else if (deferred && finishing.empty()) {
        // nothing on the GPU will free memory: wait for a release (or new work) instead of
        // retrying the admission in a busy loop
        std::unique_lock<std::mutex> lk(mu);
        cv_submit.wait_for(lk, std::chrono::milliseconds(1));
      }
      finalize_done(active.empty() && !finishing.empty());
      n_active.store((int)active.size());
      bytes_in_use.store(arena.used());
      peak_bytes.store(arena.peak());
    }
    TANQ_HIP(hipStreamSynchronize(adm_stream));
    TANQ_HIP(hipStreamSynchronize(stream));
    finalize_done(true);
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> lk(mu);
    failed = true;
    fail_msg = e.what();
    for (auto& kv : all)
      if (kv.second->state != 2) {
        kv.second->state = 2;
        kv.second->status = TANQ_E_HIP;
        kv.second->error = fail_msg;
      }
    cv_done.notify_all();
  }
}

// --------------------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------------------

namespace {

void parse_pauli_masks(int n, const char* s, std::array<uint64_t, 3>& out) {
  if (!s) fail(TANQ_E_ARG, "Pauli string is NULL");
  uint64_t xm = 0, zm = 0;
  int ny = 0, t = 0;
  for (; s[t]; ++t) {
    if (t >= n) fail(TANQ_E_ARG, "Pauli string longer than n");
    switch (s[t]) {
      case 'I': break;
      case 'X': xm |= 1ull << t; break;
      case 'Y': xm |= 1ull << t; zm |= 1ull << t; ++ny; break;
      case 'Z': zm |= 1ull << t; break;
      default: fail(TANQ_E_ARG, "bad Pauli character");
    }
  }
  if (t != n) fail(TANQ_E_ARG, "Pauli string must have exactly n characters");
  out = {xm, zm, (uint64_t)(ny & 3)};
}

void destroy_server(tanq_server_s* s) {
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_submit.notify_all();
    s->worker.join();
  }
  (void)hipSetDevice(s->device);
  if (s->adm_stream) (void)hipStreamSynchronize(s->adm_stream);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->all)
    if (kv.second->ready_ev) (void)hipEventDestroy(kv.second->ready_ev);
  for (int b = 0; b < 2; ++b) {
    if (s->graph[b]) (void)hipGraphExecDestroy(s->graph[b]);
    if (s->work_ev[b]) (void)hipEventDestroy(s->work_ev[b]);
    if (s->work_host[b]) (void)hipHostFree(s->work_host[b]);
    if (s->work_dev[b]) (void)hipFree(s->work_dev[b]);
  }
  for (auto& st : s->staged) (void)hipEventDestroy(st.ev);
  for (auto& f : s->finishing) (void)hipEventDestroy(f.ev);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->pinned_base) (void)hipHostFree(s->pinned_base);
  if (s->probs_dev) (void)hipFree(s->probs_dev);
  if (s->partials) (void)hipFree(s->partials);
  if (s->result_dev) (void)hipFree(s->result_dev);
  if (s->masks_dev) (void)hipFree(s->masks_dev);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->adm_stream) (void)hipStreamDestroy(s->adm_stream);
  delete s;
}

}  // namespace

extern "C" {

tanq_status tanq_server_create(const tanq_server_config* cfg, tanq_server* out) {
  return guarded([&] {
    if (!cfg || !out) fail(TANQ_E_ARG, "NULL argument");
    *out = nullptr;
    tanq_server_config c = *cfg;
    if (c.prec != TANQ_F32 && c.prec != TANQ_F64) fail(TANQ_E_ARG, "precision");
    if (c.max_slots < 1 || c.max_slots > 4096) fail(TANQ_E_ARG, "max_slots must be 1..4096");
    if (c.width == 0) c.width = 2;
    if (c.width != 2 && c.width != 3) fail(TANQ_E_ARG, "width must be 0, 2 or 3");
    if (c.steps_per_launch < 1 || c.steps_per_launch > 64) fail(TANQ_E_ARG, "steps_per_launch must be 1..64");
    if (c.hbm_budget < (64u << 20)) fail(TANQ_E_ARG, "hbm_budget must be at least 64 MiB");
    if (!(c.request_timeout_s >= 0.0)) fail(TANQ_E_ARG, "request_timeout_s must be >= 0");
    size_t free_b = 0, total_b = 0;
    TANQ_HIP(hipMemGetInfo(&free_b, &total_b));
    if (c.hbm_budget + (256ull << 20) > free_b) fail(TANQ_E_OOM, "hbm_budget exceeds free device memory");

    std::unique_ptr<tanq_server_s> s(new tanq_server_s);
    s->cfg = c;
    s->t0 = std::chrono::steady_clock::now();
    try {
      TANQ_HIP(hipGetDevice(&s->device));
      TANQ_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
      TANQ_HIP(hipStreamCreateWithFlags(&s->adm_stream, hipStreamNonBlocking));
      TANQ_HIP(hipMalloc((void**)&s->arena_base, c.hbm_budget));
      s->arena.init(c.hbm_budget);
      const size_t pinned_size = 256ull << 20;
      TANQ_HIP(hipHostMalloc((void**)&s->pinned_base, pinned_size, hipHostMallocDefault));
      s->pinned.init(pinned_size);
      TANQ_HIP(hipMalloc((void**)&s->probs_dev, ((size_t)1 << kServeMaxN) * sizeof(double)));
      TANQ_HIP(hipMalloc((void**)&s->partials, (size_t)reduce_partials() * sizeof(double)));
      TANQ_HIP(hipMalloc((void**)&s->result_dev, 4096 * sizeof(double)));
      TANQ_HIP(hipMalloc((void**)&s->masks_dev, 3 * 1024 * sizeof(uint64_t)));
      // chunk capacity: every slot at most kChunksPerItem chunks
      s->items_per_step = (size_t)c.max_slots;
      s->chunks_per_step = (size_t)c.max_slots * kChunksPerItem;
      s->grid = (uint64_t)std::max(1, batch_grid(c.width, (tanq_prec)c.prec));
      s->work_bytes = s->step_bytes() * c.steps_per_launch;
      for (int b = 0; b < 2; ++b) {
        TANQ_HIP(hipHostMalloc((void**)&s->work_host[b], s->work_bytes, hipHostMallocDefault));
        TANQ_HIP(hipMalloc((void**)&s->work_dev[b], s->work_bytes));
        std::memset(s->work_host[b], 0, s->work_bytes);
        TANQ_HIP(hipEventCreateWithFlags(&s->work_ev[b], hipEventDisableTiming));
      }
      if (c.use_graphs) {
        for (int b = 0; b < 2; ++b) {
          hipGraph_t gr = nullptr;
          TANQ_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
          try {
            s->record_launches(b);
          } catch (...) {
            (void)hipStreamEndCapture(s->stream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
          }
          TANQ_HIP(hipStreamEndCapture(s->stream, &gr));
          hipError_t e = hipGraphInstantiate(&s->graph[b], gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          TANQ_HIP(e);
        }
      }
      for (int i = 0; i < c.max_slots; ++i) s->free_slots.push_back(c.max_slots - 1 - i);
      s->worker = std::thread([p = s.get()] { p->loop(); });
    } catch (...) {
      destroy_server(s.release());
      throw;
    }
    *out = s.release();
  });
}

tanq_status tanq_server_submit(tanq_server s, tanq_circuit c, const tanq_outputs* outs, uint64_t* ticket) {
  return guarded([&] {
    if (!s || !c || !ticket) fail(TANQ_E_ARG, "NULL argument");
    if (c->n < s->cfg.width || c->n > kServeMaxN) fail(TANQ_E_ARG, "request qubit count outside the server's range");
    std::unique_ptr<ServeRequest> r(new ServeRequest);
    r->n = c->n;
    r->ops = c->ops;
    if (outs) {
      r->want_probs = outs->probs != 0;
      if (outs->npauli < 0 || outs->npauli > 1024) fail(TANQ_E_ARG, "npauli must be 0..1024");
      if (outs->npauli > 0 && !outs->paulis) fail(TANQ_E_ARG, "paulis is NULL");
      r->paulis.resize(outs->npauli);
      for (int i = 0; i < outs->npauli; ++i) parse_pauli_masks(c->n, outs->paulis[i], r->paulis[i]);
    }
    const tanq_prec p = (tanq_prec)s->cfg.prec;
    std::vector<PlanBlock> plan = plan_fusion(plan_ops(r->ops), r->n, s->cfg.width);
    widen_plan(plan, r->n, s->cfg.width);
    r->layout = make_fuse_layout(r->ops, plan, p);
    r->footprint = request_footprint(r->n, p, r->layout);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) fail(TANQ_E_STATE, "server failed: " + s->fail_msg);
    if (s->stop) fail(TANQ_E_STATE, "server is stopping");
    if (r->footprint > s->arena.size()) {
      ++s->n_rejected;
      fail(TANQ_E_OOM, "request footprint exceeds the server's device-memory budget");
    }
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    if (s->cfg.request_timeout_s > 0) r->deadline = r->t_submit + s->cfg.request_timeout_s;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->all[r->ticket] = std::move(r);
    ++s->n_submitted;
    s->cv_submit.notify_one();
  });
}

static void fill_result(ServeRequest* r, tanq_result* out) {
  out->status = r->status;
  out->n = r->n;
  out->trace = r->trace;
  out->probs = r->probs.empty() ? nullptr : r->probs.data();
  out->pauli = r->pauli.empty() ? nullptr : r->pauli.data();
  out->npauli = (int)r->pauli.size();
  out->fused_applies = (int)r->geom.size();
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
}

tanq_status tanq_server_poll(tanq_server s, uint64_t ticket, tanq_result* out) {
  tanq_status st = TANQ_OK;
  tanq_status rc = guarded([&] {
    if (!s || !out) fail(TANQ_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(TANQ_E_ARG, "unknown ticket");
    if (it->second->state != 2) {
      st = TANQ_E_AGAIN;
      return;
    }
    fill_result(it->second.get(), out);
  });
  return rc != TANQ_OK ? rc : st;
}

tanq_status tanq_server_wait(tanq_server s, uint64_t ticket, tanq_result* out) {
  return guarded([&] {
    if (!s || !out) fail(TANQ_E_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(TANQ_E_ARG, "unknown ticket");
    ServeRequest* r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->state == 2; });
    fill_result(r, out);
  });
}

tanq_status tanq_server_cancel(tanq_server s, uint64_t ticket) {
  return guarded([&] {
    if (!s) fail(TANQ_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(TANQ_E_ARG, "unknown ticket");
    ServeRequest* r = it->second.get();
    if (r->state == 2) return;  // finished: the result stands
    if (r->state == 0) {
      // still queued: leave the queue now
      auto q = std::find(s->pending.begin(), s->pending.end(), r);
      if (q != s->pending.end()) {
        s->pending.erase(q);
        r->status = TANQ_E_CANCELED;
        r->error = "request cancelled";
        r->t_done = s->now();
        r->state = 2;
        ++s->n_dropped;
        s->cv_done.notify_all();
        return;
      }
    }
    // admitted (or being admitted): the scheduler drops it at its next iteration
    if (r->drop == TANQ_OK) r->drop = TANQ_E_CANCELED;
  });
}

tanq_status tanq_server_release(tanq_server s, uint64_t ticket) {
  return guarded([&] {
    if (!s) fail(TANQ_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(TANQ_E_ARG, "unknown ticket");
    if (it->second->state != 2) fail(TANQ_E_STATE, "request not finished");
    s->all.erase(it);
  });
}

tanq_status tanq_server_stats_get(tanq_server s, tanq_server_stats* out) {
  return guarded([&] {
    if (!s || !out) fail(TANQ_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->n_submitted;
    out->admitted = s->n_admitted;
    out->completed = s->n_completed;
    out->rejected = s->n_rejected;
    out->launches = s->n_launches;
    out->steps = s->n_steps;
    out->bytes_in_use = s->bytes_in_use.load();
    out->peak_bytes = s->peak_bytes.load();
    out->budget_bytes = s->arena.size();
    out->active = s->n_active.load();
    out->pending = (int)s->pending.size();
    out->clock = s->now();
    out->tiles = s->n_tiles;
    out->chunks = s->n_chunks;
    out->dropped = s->n_dropped;
  });
}

tanq_status tanq_server_destroy(tanq_server s) {
  return guarded([&] {
    if (!s) return;
    destroy_server(s);
  });
}

}  // extern "C"
