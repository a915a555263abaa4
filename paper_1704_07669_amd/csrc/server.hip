// Serving runtime: many concurrent single-pass PCA streams on one GPU (see the serving section of
// include/sketch.h).
//
// Device memory (the caller's workspace) is carved once:
//   [group scratch: split partials, g operands, row-split partials of one grouped launch]
//   [zeroed arrival counters, one slice per group slot]  [device item table]
//   [finalize scratch sized for max_m x max_n]  [state arena of state_bytes]
// Each admitted stream holds Omega (FP64 and operand copy), G, H and its control block in the
// arena, placed first-fit.  Streams that do not fit wait in FIFO order.
//
// The scheduler (a library thread, or the caller through sketch_server_step) keeps at most two
// grouped launches in flight on the server stream.  A group takes the oldest pending block of up
// to max_group admitted streams, round-robin, at most one block per stream (so the H updates of a
// group never touch the same rows) and as many as fit the group scratch.  All groups are ordered on
// one stream, so the scratch is reused without waits; only the host copy of each item table is
// ringed.  Finalize runs on a second stream once the stream's blocks have completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sketch.h"
#include "common.hpp"
#include "kernels.hpp"

namespace sk {
sketch_status set_error(sketch_status st, const char* fmt, ...);
}
using namespace sk;

namespace {

constexpr int64_t kAlign = 256;
constexpr int kTableRing = 8;       // host copies of item tables in flight
constexpr int kMaxInflight = 2;     // grouped launches queued on the device at once
constexpr int kSplitsCap = 64;      // split partials of g = a Omega per item

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int op_bytes(int mode) {
  switch (mode) {
    case SKETCH_F64: return 8;
    case SKETCH_F32: return 4;
    default: return 2;
  }
}
int src_bytes(int src) { return src == SKETCH_F64 ? 8 : src == SKETCH_F32 ? 4 : 2; }
int acc_bytes(int mode) { return mode == SKETCH_F64 ? 8 : 4; }

bool src_ok(int mode, int src) {
  switch (mode) {
    case SKETCH_F64: return src == SKETCH_F64 || src == SKETCH_F32;
    case SKETCH_F32: return src == SKETCH_F32;
    case SKETCH_BF16: return src == SKETCH_F32 || src == SKETCH_BF16;
    case SKETCH_BF16X2: return src == SKETCH_F32;
    default: return false;
  }
}

const char* validate_server(const sketch_server_config* c) {
  if (!c) return "config is NULL";
  if (c->compute < SKETCH_F64 || c->compute > SKETCH_BF16X2)
    return "compute must be F64, F32, BF16 or BF16X2";
  if (!src_ok(c->compute, c->src)) return "src format not supported by the compute mode";
  if (c->l < 1 || c->l > 128) return "l must be in [1, 128]";
  if (c->max_group < 1 || c->max_group > 64) return "max_group must be in [1, 64]";
  if (c->max_n < c->l) return "max_n must be >= l";
  if (c->max_m < 1) return "max_m must be >= 1";
  if (c->max_block_rows < 1 || c->max_block_rows > (1 << 20)) return "max_block_rows out of range";
  if (c->state_bytes < 0) return "state_bytes must be >= 0";
  if (c->worker != 0 && c->worker != 1) return "worker must be 0 or 1";
  if (c->host_slots < 0 || c->host_slots > 64) return "host_slots must be in [0, 64]";
  return nullptr;
}

int src_bytes_of(int src) { return src == SKETCH_F64 ? 8 : src == SKETCH_F32 ? 4 : 2; }

struct Sizes {
  int LP, NT;
  int64_t item_bytes;     // group scratch one item may need (upper bound)
  int64_t group_bytes;    // all group slots
  int64_t cnt_per_slot;   // counters per group slot
  int64_t off_group, off_cnt, off_table, off_Q, off_Bt, off_Qb, off_tsqr, off_red,
      off_small, off_arena, off_stage, total;
  int64_t NPmax, MCAPmax, tsqr_elems, red_elems;
  int64_t LDST, stage_slot_bytes;   // staging slots for pinned-host blocks (rows padded to LDST)
};

int64_t up(int64_t v) { return rup<int64_t>(v, kAlign); }

// Upper bound of the group scratch of one block of `rows` rows and up to `n` columns.
//   split partials: splits <= 512 / row_tiles + 1 of at most kSplitsCap, so
//                   splits * rows16 <= 512 * 128 + 128 * row_tiles;
//   g operand:      LP x rows16 (hi and lo BF16, or FP32 / FP64);
//   row-split partials of a^T g: at most gemm2_partial_tiles_max() tiles.
int64_t item_bound(int64_t rows, int64_t n, int LP, int mode) {
  const int64_t rows16 = rup<int64_t>(rows, 16);
  const int64_t row_tiles = cdiv<int64_t>(rows, 128);
  // (the precision modes take at least n / kPrecCols splits)
  const int64_t split_rows = std::min<int64_t>(
      kSplitsCap * rows16, std::max<int64_t>(512 * 128 + 128 * row_tiles + 16,
                                             cdiv<int64_t>(n, kPrecCols) * rows16));
  const int g = acc_bytes(mode);
  const int64_t p1 = split_rows * LP * g;
  const int64_t gop = (int64_t)LP * rows16 * g;
  const int64_t p2 = gemm2_partial_tiles_bound(n, rows, mode) * (int64_t)LP *
                     gemm2_strip_width(mode) * g;
  return up(p1) + up(gop) + up(p2);
}

Sizes sizes(const sketch_server_config* c) {
  Sizes z{};
  z.LP = (int)rup<int64_t>(c->l, 16);
  z.NT = z.LP / 16;
  z.item_bytes = item_bound(c->max_block_rows, c->max_n, z.LP, c->compute);
  z.group_bytes = z.item_bytes * c->max_group;
  z.cnt_per_slot = rup<int64_t>(gemm2_strips(c->max_n, c->compute), 64);
  z.NPmax = rup<int64_t>(c->max_n, kNpAlign);
  z.MCAPmax = rup<int64_t>(c->max_m, 64);
  const int64_t rows_max = std::max<int64_t>(z.MCAPmax, z.NPmax);
  z.tsqr_elems = (int64_t)tsqr_workspace_elems(rows_max, 32);
  z.red_elems = (int64_t)reduce_workspace_elems(rows_max, c->l, 32);
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t r = off; off += up(bytes); return r; };
  z.off_group = take(z.group_bytes);
  z.off_cnt = take(z.cnt_per_slot * c->max_group * 4);
  z.off_table = take((int64_t)c->max_group * sizeof(PassItem));
  z.off_Q = take(z.MCAPmax * z.LP * 8);
  z.off_Bt = take(z.NPmax * z.LP * 8);
  z.off_Qb = take(z.NPmax * z.LP * 8);
  z.off_tsqr = take(z.tsqr_elems * 8);
  z.off_red = take(z.red_elems * 8);
  z.off_small = take((int64_t)finalize_small_elems(c->l, 32) * 8);
  z.off_arena = take(c->state_bytes);
  z.LDST = rup<int64_t>(c->max_n, 64);
  z.stage_slot_bytes = up(c->max_block_rows * z.LDST * src_bytes_of(c->src));
  z.off_stage = take(z.stage_slot_bytes * c->host_slots);
  z.total = off;
  return z;
}

// One stream's resident state, as offsets from the start of its arena allocation.
struct StreamLayout {
  int64_t NP, MCAP, off_om64, off_omc, off_G, off_H, off_ctrl, bytes;
};
StreamLayout stream_layout(const sketch_server_config* s, const sketch_config* c, int LP) {
  StreamLayout L{};
  L.NP = rup<int64_t>(c->n, kNpAlign);
  L.MCAP = rup<int64_t>(c->m_capacity, 64);
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t r = off; off += up(bytes); return r; };
  L.off_om64 = take(L.NP * LP * 8);
  L.off_omc = take(L.NP * LP * op_bytes(s->compute));
  L.off_G = take(L.MCAP * LP * acc_bytes(s->compute));
  L.off_H = take(L.NP * LP * 8);
  L.off_ctrl = take(sizeof(Ctrl));
  L.bytes = off;
  return L;
}

const char* validate_stream(const sketch_server_config* s, const sketch_config* c) {
  if (!c) return "config is NULL";
  if (c->n < 1 || c->n > s->max_n) return "n must be in [1, max_n]";
  if (c->m_capacity < 1 || c->m_capacity > s->max_m) return "m_capacity must be in [1, max_m]";
  if (c->max_block_rows < 1 || c->max_block_rows > s->max_block_rows)
    return "max_block_rows must be in [1, the server's max_block_rows]";
  if (c->l != s->l) return "l must equal the server's l";
  if (c->compute != s->compute) return "compute must equal the server's compute";
  if (c->k < 1 || c->k > c->l) return "k must be in [1, l]";
  if (c->b < 1 || c->b > 32 || c->l % c->b != 0) return "b must be in [1, 32] and divide l";
  if (c->l > c->n) return "l must be <= n";
  if (c->omega_from_seed != 1) return "served streams draw Omega from their seed";
  if (c->host_slots != 0) return "served streams take device rows (host_slots = 0)";
  if (c->centre != 0) return "served streams are not centred (centre = 0)";
  if (c->want_u != 0 && c->want_u != 1) return "want_u must be 0 or 1";
  return nullptr;
}

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  void reset(int64_t size) { free_.clear(); if (size > 0) free_[0] = size; used_ = 0; peak_ = 0; }
  bool alloc(int64_t bytes, int64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const int64_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest > 0) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(int64_t off, int64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
    used_ -= bytes;
  }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t used_ = 0, peak_ = 0;
};

struct Block {
  const void* rows;
  int64_t nrows, ld;
  uint64_t ticket;
  double t_submit;         // arrival time the latency is measured from (host clock)
  bool host;               // pinned host rows, copied into a staging slot at launch
};

enum { S_QUEUED = 0, S_ACTIVE = 1, S_FINALIZING = 2 };

struct Stream {
  uint64_t id;
  sketch_config cfg;
  StreamLayout lay;
  int state = S_QUEUED;
  int64_t arena_off = -1;
  int64_t rows_submitted = 0;   // capacity check
  int64_t rows_launched = 0;    // first G row of the next launched block
  std::deque<Block> pending;
  int inflight = 0;             // launched blocks not yet retired
  bool closing = false;         // finalize requested: no more submits
};

struct Group {
  hipEvent_t ev;
  int table_slot;
  std::vector<std::pair<uint64_t, uint64_t>> blocks;   // (stream id, ticket)
  std::vector<double> t_submit;
  std::vector<int> stage_slots;                        // staging slots its host blocks hold
};

}  // namespace

struct sketch_server_s {
  sketch_server_config cfg;
  Sizes z;
  uint8_t* ws = nullptr;
  hipStream_t stream = nullptr;      // grouped launches (caller's)
  hipStream_t fin_stream = nullptr;  // finalize (library's)
  void* fin_pin = nullptr;           // pinned staging of the finalize's read-backs
  hipEvent_t fin_ev = nullptr;       // the event those read-backs poll
  hipStream_t copy_stream = nullptr; // host-to-device copies of pinned-host blocks (library's)
  std::vector<char> stage_busy;      // staging slots held by an in-flight group
  std::vector<hipEvent_t> stage_ev;  // per slot: its copy finished
  int device = 0;
  sketch_status sticky = SKETCH_OK;

  std::mutex mu;                     // everything below
  std::condition_variable cv_work;   // worker wake-up
  std::condition_variable cv_done;   // groups retired / streams released
  Arena arena;
  uint64_t next_id = 1, next_ticket = 1;
  std::unordered_map<uint64_t, Stream> streams;
  std::deque<uint64_t> waitq;        // queued stream ids, FIFO
  std::vector<uint64_t> order;       // admitted stream ids, round-robin order
  size_t rr = 0;
  std::deque<Group> inflight;
  std::vector<hipEvent_t> ev_pool;
  PassItem* host_tables = nullptr;   // kTableRing x max_group, pinned
  hipEvent_t table_ev[kTableRing] = {};
  bool table_used[kTableRing] = {};
  int next_table = 0;
  std::vector<std::pair<uint64_t, double>> done;   // (ticket, latency)
  hipEvent_t anchor = nullptr;       // recorded on the idle launch stream at host time t_anchor
  double t_anchor = 0.0;
  sketch_server_stats st{};

  std::mutex fin_mu;                 // the finalize scratch
  std::thread worker;
  bool stop = false;

  template <typename T> T* at(int64_t off) { return reinterpret_cast<T*>(ws + off); }

  sketch_status dev_fail(hipError_t e, const char* what) {
    sticky = SKETCH_E_DEVICE;
    return set_error(SKETCH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }
};

namespace {

sketch_status check_server(sketch_server_t s) {
  if (!s) return set_error(SKETCH_E_INVAL, "server is NULL");
  if (s->sticky != SKETCH_OK)
    return set_error(s->sticky, "server is in a sticky error state (%d)", (int)s->sticky);
  return SKETCH_OK;
}

// Places and initialises a stream's state (Alg. 4 steps 1-3): Omega from the seed rounded to the
// operand format, H = 0, control block cleared.  Caller holds mu.
sketch_status admit_locked(sketch_server_t s, Stream& st) {
  int64_t off = 0;
  if (!s->arena.alloc(st.lay.bytes, &off)) return SKETCH_E_CAPACITY;
  st.arena_off = off;
  uint8_t* base = s->ws + s->z.off_arena + off;
  const StreamLayout& L = st.lay;
  double* om64 = reinterpret_cast<double*>(base + L.off_om64);
  hipError_t e = launch_omega_philox(st.cfg.seed, st.cfg.n, st.cfg.l, om64, L.NP, s->stream);
  if (e == hipSuccess)
    e = launch_omega_quantize(s->cfg.compute, st.cfg.n, L.NP, st.cfg.l, s->z.LP, om64,
                              base + L.off_omc, s->stream);
  if (e == hipSuccess)
    e = launch_fill_f64(reinterpret_cast<double*>(base + L.off_H), L.NP * s->z.LP, 0.0, s->stream);
  if (e == hipSuccess)
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(base + L.off_ctrl), sizeof(Ctrl) / 4, 0u,
                        s->stream);
  if (e != hipSuccess) return s->dev_fail(e, "stream admission");
  st.state = S_ACTIVE;
  s->order.push_back(st.id);
  return SKETCH_OK;
}

sketch_status admit_waiting_locked(sketch_server_t s) {
  while (!s->waitq.empty()) {
    Stream& st = s->streams.at(s->waitq.front());
    sketch_status r = admit_locked(s, st);
    if (r == SKETCH_E_CAPACITY) break;   // FIFO: later streams wait behind the head
    if (r != SKETCH_OK) return r;
    s->waitq.pop_front();
  }
  return SKETCH_OK;
}

// Retires finished groups (in launch order).  Caller holds mu.
sketch_status retire_locked(sketch_server_t s) {
  bool any = false;
  while (!s->inflight.empty()) {
    Group& g = s->inflight.front();
    hipError_t e = hipEventQuery(g.ev);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return s->dev_fail(e, "group completion");
    // the group's completion time on the GPU, in host time through the anchor event
    float ms = 0.f;
    double t = now_s();
    if (s->anchor && hipEventElapsedTime(&ms, s->anchor, g.ev) == hipSuccess)
      t = s->t_anchor + 1e-3 * (double)ms;
    else
      (void)hipGetLastError();
    for (size_t i = 0; i < g.blocks.size(); ++i) {
      auto it = s->streams.find(g.blocks[i].first);
      if (it != s->streams.end()) it->second.inflight--;
      s->done.push_back({g.blocks[i].second, t - g.t_submit[i]});
    }
    for (int sl : g.stage_slots) s->stage_busy[sl] = 0;
    s->ev_pool.push_back(g.ev);
    s->inflight.pop_front();
    any = true;
  }
  // refresh the anchor while the stream is idle, so the float milliseconds of the event
  // intervals stay fine-grained
  if (any && s->inflight.empty() && s->anchor && now_s() - s->t_anchor > 10.0) {
    hipError_t e = hipEventRecord(s->anchor, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->anchor);
    if (e != hipSuccess) return s->dev_fail(e, "latency anchor");
    s->t_anchor = now_s();
  }
  if (any) s->cv_done.notify_all();
  return SKETCH_OK;
}

// Forms and launches one group.  Caller holds mu.
sketch_status launch_group_locked(sketch_server_t s, int32_t* launched) {
  *launched = 0;
  if ((int)s->inflight.size() >= kMaxInflight || s->order.empty()) return SKETCH_OK;
  const sketch_server_config& c = s->cfg;
  const Sizes& z = s->z;
  const int slot = s->next_table;
  if (s->table_used[slot]) {
    hipError_t e = hipEventQuery(s->table_ev[slot]);
    if (e == hipErrorNotReady) return SKETCH_OK;
    if (e != hipSuccess) return s->dev_fail(e, "item table reuse");
  }
  PassItem* items = s->host_tables + (int64_t)slot * c.max_group;
  Group g{};
  int count = 0;
  int64_t scratch = 0;
  const size_t nord = s->order.size();
  size_t visited = 0;
  for (; visited < nord && count < c.max_group; ++visited) {
    const uint64_t id = s->order[(s->rr + visited) % nord];
    Stream& st = s->streams.at(id);
    if (st.pending.empty()) continue;
    const Block& bk = st.pending.front();
    // a pinned-host block needs a free staging slot; without one it waits for a later group
    int stage = -1;
    if (bk.host) {
      for (int i = 0; i < c.host_slots; ++i)
        if (!s->stage_busy[i]) { stage = i; break; }
      if (stage < 0) continue;
    }
    uint8_t* base = s->ws + z.off_arena + st.arena_off;
    uint8_t* grp = s->ws + z.off_group + scratch;
    PassItem it{};
    it.A = bk.rows;
    it.lda = bk.ld;
    if (bk.host) {
      it.A = s->ws + z.off_stage + (int64_t)stage * z.stage_slot_bytes;
      it.lda = z.LDST;
    }
    it.nrows = (int)bk.nrows;
    it.n = st.cfg.n;
    it.omc = base + st.lay.off_omc;
    it.NP = st.lay.NP;
    it.ldp = rup<int64_t>(bk.nrows, 16);
    it.G = base + st.lay.off_G;
    it.ldg = st.lay.MCAP;
    it.g_row0 = st.rows_launched;
    it.H = reinterpret_cast<double*>(base + st.lay.off_H);
    it.ldh = st.lay.NP;
    it.fp8_exp = nullptr;
    it.ctrl = reinterpret_cast<Ctrl*>(base + st.lay.off_ctrl);
    it.counters = s->at<unsigned>(z.off_cnt) + (int64_t)count * z.cnt_per_slot;
    plan_item(it, c.compute, c.src, (int)std::min<int64_t>(kSplitsCap, st.lay.NP / kNpAlign));
    const int g8 = acc_bytes(c.compute);
    const int64_t p1 = up((int64_t)it.splits * z.LP * it.ldp * g8);
    const int64_t gop = up((int64_t)z.LP * it.ldp * g8);
    const int64_t p2 = it.rsplit > 1
        ? up((int64_t)it.strips * it.rsplit * z.LP * gemm2_strip_width(c.compute) * g8) : 0;
    if (scratch + p1 + gop + p2 > z.group_bytes) break;   // the group is full
    if (bk.host) {
      // copy on the library's copy stream; the grouped launch waits for it
      const int es = src_bytes_of(c.src);
      hipError_t e = hipMemcpy2DAsync(const_cast<void*>(it.A), z.LDST * es, bk.rows, bk.ld * es,
                                      st.cfg.n * es, bk.nrows, hipMemcpyHostToDevice,
                                      s->copy_stream);
      if (e == hipSuccess) e = hipEventRecord(s->stage_ev[stage], s->copy_stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->stage_ev[stage], 0);
      if (e != hipSuccess) return s->dev_fail(e, "host block copy");
      s->stage_busy[stage] = 1;
      g.stage_slots.push_back(stage);
    }
    it.P1 = grp;
    it.Gop = grp + p1;
    it.P2 = (it.rsplit > 1) ? (void*)(grp + p1 + gop) : nullptr;
    scratch += p1 + gop + p2;
    items[count++] = it;
    st.rows_launched += bk.nrows;
    st.inflight++;
    g.blocks.push_back({id, bk.ticket});
    g.t_submit.push_back(bk.t_submit);
    st.pending.pop_front();
  }
  if (count == 0) return SKETCH_OK;
  s->rr = (s->rr + visited) % nord;

  PassGroup pg{};
  pg.mode = c.compute;
  pg.src = c.src;
  pg.LP = z.LP;
  pg.NT = z.NT;
  plan_group(pg, items, count);
  hipError_t e = hipSuccess;
  if (count > 1) {
    PassItem* dev = s->at<PassItem>(z.off_table);
    e = hipMemcpyAsync(dev, items, (size_t)count * sizeof(PassItem), hipMemcpyHostToDevice,
                       s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->table_ev[slot], s->stream);
    s->table_used[slot] = true;
    s->next_table = (slot + 1) % kTableRing;
    pg.dev = dev;
  }
  if (e == hipSuccess) e = launch_gemm1(pg, s->stream);
  if (e == hipSuccess) e = launch_reduce1(pg, s->stream);
  if (e == hipSuccess) e = launch_gemm2(pg, s->stream);
  if (e == hipSuccess) {
    if (s->ev_pool.empty()) {
      hipEvent_t ev;
      e = hipEventCreate(&ev);          // timed: its timestamp gives the blocks' latency
      if (e == hipSuccess) s->ev_pool.push_back(ev);
    }
  }
  if (e == hipSuccess) {
    g.ev = s->ev_pool.back();
    s->ev_pool.pop_back();
    e = hipEventRecord(g.ev, s->stream);
  }
  if (e != hipSuccess) return s->dev_fail(e, "grouped launch");
  g.table_slot = slot;
  s->inflight.push_back(std::move(g));
  s->st.groups++;
  s->st.blocks += count;
  s->st.max_blocks_in_group = std::max<int64_t>(s->st.max_blocks_in_group, count);
  *launched = count;
  return SKETCH_OK;
}

sketch_status step_locked(sketch_server_t s, int32_t* launched) {
  sketch_status r = retire_locked(s);
  if (r == SKETCH_OK) r = admit_waiting_locked(s);
  if (r == SKETCH_OK) r = launch_group_locked(s, launched);
  return r;
}

bool has_work_locked(sketch_server_t s) {
  for (uint64_t id : s->order)
    if (!s->streams.at(id).pending.empty()) return true;
  return !s->inflight.empty();
}

void worker_main(sketch_server_t s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    if (s->sticky != SKETCH_OK) {
      s->cv_done.notify_all();
      s->cv_work.wait(lk, [&] { return s->stop; });
      break;
    }
    int32_t launched = 0;
    step_locked(s, &launched);
    if (launched > 0) continue;
    if (!s->inflight.empty()) {
      // poll the oldest group briefly without holding the lock
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (!has_work_locked(s)) {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

}  // namespace

extern "C" {

size_t sketch_server_workspace_size(const sketch_server_config* cfg) {
  if (const char* why = validate_server(cfg)) {
    set_error(SKETCH_E_INVAL, "%s", why);
    return 0;
  }
  return (size_t)sizes(cfg).total;
}

size_t sketch_server_stream_bytes(const sketch_server_config* srv, const sketch_config* cfg) {
  if (const char* why = validate_server(srv)) {
    set_error(SKETCH_E_INVAL, "%s", why);
    return 0;
  }
  if (const char* why = validate_stream(srv, cfg)) {
    set_error(SKETCH_E_INVAL, "%s", why);
    return 0;
  }
  return (size_t)stream_layout(srv, cfg, (int)rup<int64_t>(srv->l, 16)).bytes;
}

sketch_status sketch_server_create(sketch_server_t* out, const sketch_server_config* cfg,
                                   void* dev_ws, size_t ws_bytes, void* hip_stream) {
  if (!out) return set_error(SKETCH_E_INVAL, "out is NULL");
  *out = nullptr;
  if (const char* why = validate_server(cfg)) return set_error(SKETCH_E_INVAL, "%s", why);
  const Sizes z = sizes(cfg);
  if (!dev_ws) return set_error(SKETCH_E_INVAL, "workspace is NULL");
  if (((uintptr_t)dev_ws) % kAlign) return set_error(SKETCH_E_INVAL, "workspace must be 256-byte aligned");
  if ((int64_t)ws_bytes < z.total)
    return set_error(SKETCH_E_NOMEM, "workspace holds %zu bytes, %lld needed", ws_bytes,
                     (long long)z.total);
  hipError_t e = finalize_prepare();
  if (e != hipSuccess) return set_error(SKETCH_E_DEVICE, "kernel attributes: %s", hipGetErrorString(e));
  sketch_server_s* s = new sketch_server_s();
  s->cfg = *cfg;
  s->z = z;
  s->ws = (uint8_t*)dev_ws;
  s->stream = (hipStream_t)hip_stream;
  s->arena.reset(cfg->state_bytes);
  e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->fin_stream, hipStreamNonBlocking);
  if (e == hipSuccess && cfg->host_slots > 0)
    e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
  s->stage_busy.assign(cfg->host_slots, 0);
  s->stage_ev.assign(cfg->host_slots, nullptr);
  for (int i = 0; i < cfg->host_slots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&s->stage_ev[i], hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->host_tables,
                      sizeof(PassItem) * (size_t)kTableRing * cfg->max_group, hipHostMallocDefault);
  for (int i = 0; i < kTableRing && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&s->table_ev[i], hipEventDisableTiming);
  if (e == hipSuccess)
    e = launch_fill_u32(s->at<uint32_t>(z.off_cnt), z.cnt_per_slot * cfg->max_group, 0u, s->stream);
  // the finalize's small matrices start defined (no kernel reads them before writing, but a
  // rejected factorisation must never meet uninitialised memory)
  if (e == hipSuccess)
    e = launch_fill_f64(s->at<double>(z.off_small), (int64_t)finalize_small_elems(cfg->l, 32), 0.0,
                        s->stream);
  if (e == hipSuccess) e = hipHostMalloc(&s->fin_pin, kHostPinBytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fin_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&s->anchor);
  if (e == hipSuccess) e = hipEventRecord(s->anchor, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  s->t_anchor = now_s();
  if (e != hipSuccess) {
    const char* msg = hipGetErrorString(e);
    s->sticky = SKETCH_E_DEVICE;
    sketch_server_destroy(s);
    return set_error(SKETCH_E_DEVICE, "server creation: %s", msg);
  }
  if (cfg->worker) s->worker = std::thread(worker_main, s);
  *out = s;
  return SKETCH_OK;
}

sketch_status sketch_server_open(sketch_server_t s, const sketch_config* cfg, uint64_t* stream_id,
                                 int32_t* admitted) {
  if (sketch_status r = check_server(s)) return r;
  if (!stream_id) return set_error(SKETCH_E_INVAL, "stream_id is NULL");
  if (const char* why = validate_stream(&s->cfg, cfg)) return set_error(SKETCH_E_INVAL, "%s", why);
  Stream st;
  st.cfg = *cfg;
  st.lay = stream_layout(&s->cfg, cfg, s->z.LP);
  if (st.lay.bytes > s->cfg.state_bytes)
    return set_error(SKETCH_E_CAPACITY, "stream state (%lld bytes) exceeds the state budget",
                     (long long)st.lay.bytes);
  std::lock_guard<std::mutex> lk(s->mu);
  st.id = s->next_id++;
  const uint64_t id = st.id;
  s->streams.emplace(id, st);
  s->waitq.push_back(id);
  s->st.queued_peak = std::max<int64_t>(s->st.queued_peak, (int64_t)s->waitq.size());
  sketch_status r = admit_waiting_locked(s);
  if (r != SKETCH_OK) return r;
  *stream_id = id;
  if (admitted) *admitted = (s->streams.at(id).state == S_ACTIVE);
  s->cv_work.notify_one();
  return SKETCH_OK;
}

sketch_status sketch_server_submit(sketch_server_t s, uint64_t stream_id, const void* rows,
                                   int64_t nrows, int64_t ld, uint64_t* ticket) {
  return sketch_server_submit_ex(s, stream_id, rows, 1, nrows, ld, -1.0, ticket);
}

double sketch_server_clock(void) { return now_s(); }

sketch_status sketch_server_submit_ex(sketch_server_t s, uint64_t stream_id, const void* rows,
                                      int32_t src_is_device, int64_t nrows, int64_t ld,
                                      double arrival_s, uint64_t* ticket) {
  if (sketch_status r = check_server(s)) return r;
  if (!rows) return set_error(SKETCH_E_INVAL, "rows is NULL");
  if (src_is_device != 0 && src_is_device != 1)
    return set_error(SKETCH_E_INVAL, "src_is_device must be 0 or 1");
  if (!src_is_device) {
    if (s->cfg.host_slots == 0) return set_error(SKETCH_E_INVAL, "server has no host staging slots");
    hipPointerAttribute_t at;
    memset(&at, 0, sizeof(at));
    if (hipPointerGetAttributes(&at, rows) != hipSuccess || at.type != hipMemoryTypeHost) {
      (void)hipGetLastError();
      return set_error(SKETCH_E_INVAL, "host rows must be pinned (hipHostMalloc)");
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->streams.find(stream_id);
  if (it == s->streams.end()) return set_error(SKETCH_E_INVAL, "unknown stream %llu", (unsigned long long)stream_id);
  Stream& st = it->second;
  if (st.closing) return set_error(SKETCH_E_STATE, "stream is being finalized");
  if (nrows < 1) return set_error(SKETCH_E_INVAL, "nrows must be >= 1");
  if (ld < st.cfg.n) return set_error(SKETCH_E_INVAL, "ld must be >= n");
  if (nrows > st.cfg.max_block_rows)
    return set_error(SKETCH_E_CAPACITY, "block of %lld rows exceeds max_block_rows", (long long)nrows);
  if (st.rows_submitted + nrows > st.cfg.m_capacity)
    return set_error(SKETCH_E_CAPACITY, "m_capacity %lld exceeded", (long long)st.cfg.m_capacity);
  const uint64_t tk = s->next_ticket++;
  st.pending.push_back({rows, nrows, ld, tk, arrival_s >= 0.0 ? arrival_s : now_s(),
                        src_is_device == 0});
  st.rows_submitted += nrows;
  if (ticket) *ticket = tk;
  s->cv_work.notify_one();
  return SKETCH_OK;
}

sketch_status sketch_server_step(sketch_server_t s, int32_t* launched) {
  if (sketch_status r = check_server(s)) return r;
  if (s->cfg.worker) return set_error(SKETCH_E_STATE, "the server runs its own scheduler");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t n = 0;
  sketch_status r = step_locked(s, &n);
  if (launched) *launched = n;
  return r;
}

sketch_status sketch_server_poll(sketch_server_t s, uint64_t* tickets, double* latency_s,
                                 int32_t cap, int32_t* count) {
  if (sketch_status r = check_server(s)) return r;
  if (!count || cap < 0 || (cap > 0 && (!tickets || !latency_s)))
    return set_error(SKETCH_E_INVAL, "bad output arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->cfg.worker) {
    sketch_status r = retire_locked(s);
    if (r != SKETCH_OK) return r;
  }
  const int32_t n = (int32_t)std::min<size_t>((size_t)cap, s->done.size());
  for (int32_t i = 0; i < n; ++i) {
    tickets[i] = s->done[i].first;
    latency_s[i] = s->done[i].second;
  }
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *count = n;
  return SKETCH_OK;
}

sketch_status sketch_server_finalize(sketch_server_t s, uint64_t stream_id, double* S_dev,
                                     double* U_dev, int64_t ldu, double* V_dev, int64_t ldv,
                                     int32_t* rank_out) {
  if (sketch_status r = check_server(s)) return r;
  if (!S_dev || !V_dev) return set_error(SKETCH_E_INVAL, "S and V are required");
  Stream st;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end()) return set_error(SKETCH_E_INVAL, "unknown stream %llu", (unsigned long long)stream_id);
    Stream& ref = it->second;
    if (ref.closing) return set_error(SKETCH_E_STATE, "stream is already being finalized");
    if (ref.state == S_QUEUED)
      return set_error(SKETCH_E_STATE, "stream is still waiting for memory; finalize others first");
    if (ldv < ref.cfg.k) return set_error(SKETCH_E_INVAL, "ldv must be >= k");
    if (U_dev && (!ref.cfg.want_u || ldu < ref.cfg.k))
      return set_error(SKETCH_E_INVAL, "U needs want_u = 1 and ldu >= k");
    ref.closing = true;
    // every block of the stream launched and completed (the stream must first be admitted)
    for (;;) {
      Stream& cur = s->streams.at(stream_id);
      if (s->sticky != SKETCH_OK) return set_error(s->sticky, "server failed");
      if (cur.state == S_ACTIVE && cur.pending.empty() && cur.inflight == 0) break;
      if (s->cfg.worker) {
        s->cv_work.notify_one();
        s->cv_done.wait_for(lk, std::chrono::milliseconds(1));
      } else {
        int32_t n = 0;
        sketch_status r = step_locked(s, &n);
        if (r != SKETCH_OK) return r;
        if (n == 0 && !s->inflight.empty()) {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
        }
      }
    }
    Stream& cur = s->streams.at(stream_id);
    cur.state = S_FINALIZING;
    st = cur;
  }
  sketch_status result = SKETCH_OK;
  int32_t rank = 0;
  {
    std::lock_guard<std::mutex> fk(s->fin_mu);
    const Sizes& z = s->z;
    uint8_t* base = s->ws + z.off_arena + st.arena_off;
    const sketch_config& c = st.cfg;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + st.lay.off_ctrl);
    hipError_t e = hipSuccess;
    if (st.rows_launched == 0) {
      e = launch_fill_f64(S_dev, c.k, 0.0, s->fin_stream);
      if (e == hipSuccess) e = launch_fill_rows(V_dev, c.n, c.k, ldv, 0.0, s->fin_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->fin_stream);
    } else {
      FinalizeArgs f{};
      f.mode = s->cfg.compute;
      f.m = st.rows_launched;
      f.n = c.n;
      f.k = c.k;
      f.l = c.l;
      f.b = c.b;
      f.LP = z.LP;
      f.G = base + st.lay.off_G;
      f.ldg = st.lay.MCAP;
      f.H = reinterpret_cast<double*>(base + st.lay.off_H);
      f.ldh = st.lay.NP;
      f.om64 = reinterpret_cast<double*>(base + st.lay.off_om64);
      f.ldo = st.lay.NP;
      f.Q = s->at<double>(z.off_Q);
      f.ldq = st.lay.MCAP;
      f.Bt = s->at<double>(z.off_Bt);
      f.Qb = s->at<double>(z.off_Qb);
      f.ldb = st.lay.NP;
      f.tsqr_ws = s->at<double>(z.off_tsqr);
      f.tsqr_ws_elems = z.tsqr_elems;
      f.red_ws = s->at<double>(z.off_red);
      f.red_ws_elems = z.red_elems;
      f.small = s->at<double>(z.off_small);
      f.ctrl = ctrl;
      f.S = S_dev;
      f.U = U_dev;
      f.ldu = ldu;
      f.V = V_dev;
      f.ldv = ldv;
      f.host_pin = s->fin_pin;
      f.host_ev = s->fin_ev;
      Ctrl hc{};
      f.ctrl_host = &hc;
      e = run_finalize(f, s->fin_stream);
      if (e == hipSuccess && !f.ctrl_read)
        e = read_back(&hc, ctrl, sizeof(Ctrl), s->fin_stream, s->fin_pin, s->fin_ev);
      if (e == hipSuccess) {
        rank = hc.l_eff;
        if (hc.nonfinite) result = set_error(SKETCH_E_NONFINITE, "a block of the stream held NaN or Inf");
      }
    }
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      return s->dev_fail(e, "stream finalize");
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->arena.release(st.arena_off, st.lay.bytes);
    s->order.erase(std::find(s->order.begin(), s->order.end(), stream_id));
    if (s->rr >= s->order.size()) s->rr = 0;
    s->streams.erase(stream_id);
    s->st.finalized++;
    sketch_status r = admit_waiting_locked(s);
    s->cv_work.notify_one();
    if (r != SKETCH_OK) return r;
  }
  if (rank_out) *rank_out = rank;
  return result;
}

sketch_status sketch_server_get_stats(sketch_server_t s, sketch_server_stats* out) {
  if (!s || !out) return set_error(SKETCH_E_INVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  int64_t active = 0;
  for (auto& kv : s->streams)
    if (kv.second.state != S_QUEUED) active++;
  out->active = active;
  out->queued = (int64_t)s->waitq.size();
  out->state_used = s->arena.used();
  out->state_peak = s->arena.peak();
  return SKETCH_OK;
}

sketch_status sketch_server_destroy(sketch_server_t s) {
  if (!s) return set_error(SKETCH_E_INVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->fin_stream) {
    (void)hipStreamSynchronize(s->fin_stream);
    (void)hipStreamDestroy(s->fin_stream);
  }
  for (auto& g : s->inflight) (void)hipEventDestroy(g.ev);
  for (auto ev : s->ev_pool) (void)hipEventDestroy(ev);
  if (s->anchor) (void)hipEventDestroy(s->anchor);
  if (s->fin_pin) (void)hipHostFree(s->fin_pin);
  if (s->fin_ev) (void)hipEventDestroy(s->fin_ev);
  for (auto ev : s->stage_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (s->copy_stream) {
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipStreamDestroy(s->copy_stream);
  }
  for (int i = 0; i < kTableRing; ++i)
    if (s->table_ev[i]) (void)hipEventDestroy(s->table_ev[i]);
  if (s->host_tables) (void)hipHostFree(s->host_tables);
  delete s;
  return SKETCH_OK;
}

}  // extern "C"
