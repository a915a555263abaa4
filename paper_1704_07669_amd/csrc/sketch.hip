// Runtime and C ABI of the single-pass PCA library (see include/sketch.h).
//
// Device state lives in the caller's workspace, carved here.  All kernels run on the caller's
// stream; pinned-host blocks are copied on a library-owned side stream into a ring of device
// staging slots, with events ordering copy -> compute and compute -> reuse of the slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sketch.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace sk;

namespace {

thread_local std::string g_err;

}  // namespace

namespace sk {
sketch_status set_error(sketch_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
}  // namespace sk

namespace {

#define fail sk::set_error

constexpr int kRing = 16;          // per-ticket completion events
constexpr int64_t kAlign = 256;    // workspace carve alignment (bytes)
constexpr int kMaxSplits = 64;

int src_size(int dt) {
  switch (dt) {
    case SKETCH_F64: return 8;
    case SKETCH_F32: return 4;
    case SKETCH_BF16: return 2;
    default: return 0;
  }
}

bool mode_accepts(int mode, int src) {
  switch (mode) {
    case SKETCH_F64: return src == SKETCH_F64 || src == SKETCH_F32;
    case SKETCH_F32: return src == SKETCH_F32;
    case SKETCH_BF16: return src == SKETCH_F32 || src == SKETCH_BF16;
    case SKETCH_BF16X2: return src == SKETCH_F32;
    case SKETCH_FP8_E4M3: return src == SKETCH_F32;
    default: return false;
  }
}

int op_size(int mode) {
  switch (mode) {
    case SKETCH_F64: return 8;
    case SKETCH_F32: return 4;
    case SKETCH_BF16:
    case SKETCH_BF16X2: return 2;
    default: return 1;
  }
}

struct Layout {
  int LP, NT, t, splits_max;
  int64_t NP, MCAP, RBP, LDST, NQ;
  int64_t off_ctrl, off_fp8, off_om64, off_omc, off_G, off_H, off_P1, off_Gop, off_P2, off_cnt, off_stage, off_fp8q,
      off_Q, off_Q2, off_Bt, off_Qb, off_tsqr, off_red, off_small, off_mu, total;
  int64_t stage_slot_bytes;
  int64_t tsqr_elems, red_elems;
};

const char* validate(const sketch_config* c) {
  if (!c) return "config is NULL";
  if (c->n < 1) return "n must be >= 1";
  if (c->m_capacity < 1) return "m_capacity must be >= 1";
  if (c->max_block_rows < 1) return "max_block_rows must be >= 1";
  if (c->max_block_rows > (int64_t)1 << 30) return "max_block_rows too large";
  if (c->l < 1 || c->l > 128) return "l must be in [1, 128]";
  if (c->k < 1 || c->k > c->l) return "k must be in [1, l]";
  if (c->b < 1 || (c->b > 32 && c->b != c->l) || c->l % c->b != 0)
    return "b must divide l and be in [1, 32] or equal l";
  if (c->l > c->n) return "l must be <= n";
  if (c->compute < SKETCH_F64 || c->compute > SKETCH_FP8_E4M3) return "unknown compute mode";
  if (c->host_slots != 0 && (c->host_slots < 2 || c->host_slots > 4))
    return "host_slots must be 0 or 2..4";
  if (c->host_slots > 0 && !mode_accepts(c->compute, c->host_src))
    return "host_src not supported by the compute mode";
  if (c->want_u != 0 && c->want_u != 1) return "want_u must be 0 or 1";
  if (c->omega_from_seed != 0 && c->omega_from_seed != 1) return "omega_from_seed must be 0 or 1";
  if (c->centre != 0 && c->centre != 1) return "centre must be 0 or 1";
  if (c->centre && c->l > 127) return "l must be <= 127 with centre = 1";
  if (c->reserved != 0) return "reserved must be 0";
  return nullptr;
}

Layout plan(const sketch_config* c) {
  Layout L{};
  L.LP = (int)rup<int64_t>(c->l + (c->centre ? 1 : 0), 16);   // the column sums take column l
  L.NT = L.LP / 16;
  L.t = c->l / c->b;
  L.NP = rup<int64_t>(c->n, kNpAlign);
  L.MCAP = rup<int64_t>(c->m_capacity, 64);
  L.RBP = rup<int64_t>(c->max_block_rows, 16);
  L.splits_max = (int)std::min<int64_t>(kMaxSplits, L.NP / kNpAlign);
  L.LDST = rup<int64_t>(c->n, 64);
  L.NQ = rup<int64_t>(c->n, kNpAlign);
  const int gsz = (c->compute == SKETCH_F64) ? 8 : 4;
  L.stage_slot_bytes =
      c->host_slots > 0 ? rup<int64_t>(c->max_block_rows * L.LDST * src_size(c->host_src), kAlign)
                        : 0;
  const int64_t rows_max = std::max<int64_t>(L.MCAP, L.NP);
  L.tsqr_elems = (int64_t)tsqr_workspace_elems(rows_max, std::min(c->b, 32));
  L.red_elems = (int64_t)reduce_workspace_elems(rows_max, c->l, c->b);
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t r = off; off += rup<int64_t>(bytes, kAlign); return r; };
  L.off_ctrl = take(sizeof(Ctrl));
  L.off_fp8 = take(64);
  L.off_om64 = take((int64_t)L.LP * L.NP * 8);
  L.off_omc = take((int64_t)L.LP * L.NP * op_size(c->compute));
  L.off_G = take((int64_t)L.LP * L.MCAP * gsz);
  L.off_H = take((int64_t)L.LP * L.NP * 8);
  L.off_P1 = take((int64_t)L.splits_max * L.LP * L.RBP * gsz);
  L.off_Gop = take((int64_t)L.LP * L.RBP * gsz);
  L.off_P2 = take(gemm2_strips(c->n, c->compute) * kGemm2MaxSplits * L.LP *
                  gemm2_strip_width(c->compute) * gsz);
  L.off_cnt = take(gemm2_strips(c->n, c->compute) * 4);
  L.off_stage = take(L.stage_slot_bytes * c->host_slots);
  L.off_fp8q = take(c->compute == SKETCH_FP8_E4M3 ? c->max_block_rows * L.NQ : 0);
  L.off_Q = take((int64_t)L.LP * L.MCAP * 8);
  L.off_Q2 = take(c->b == c->l ? (int64_t)L.LP * L.MCAP * 8 : 0);   // one-block finalize
  L.off_Bt = take((int64_t)L.LP * L.NP * 8);
  L.off_Qb = take((int64_t)L.LP * L.NP * 8);
  L.off_tsqr = take(L.tsqr_elems * 8);
  L.off_red = take(L.red_elems * 8);
  L.off_small = take((int64_t)finalize_small_elems(c->l, c->b) * 8);
  L.off_mu = take(c->centre ? L.NP * 8 : 0);
  L.total = off;
  return L;
}

}  // namespace

struct sketch_s {
  sketch_config cfg;
  Layout lay;
  uint8_t* ws = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t copy = nullptr;
  int device = 0;
  // state
  int64_t rows = 0;
  int phase = 0;                    // 0: needs Omega, 1: ingesting, 2: finalized
  sketch_status sticky = SKETCH_OK;
  int* nf_host = nullptr;           // host-mapped non-finite flag (host address), or null
  int* nf_dev = nullptr;            // its device address
  void* fin_pin = nullptr;          // pinned staging of the finalize's read-backs, or null
  hipEvent_t fin_ev = nullptr;      // the event those read-backs poll, or null
  int32_t path_loop = -1, path_rb = -1;   // QR methods the last finalize used
  int32_t force_loop = 0, force_rb = 0;   // test hook: take the Householder paths directly
  bool omega_derived = false;       // Omega' came from the data (power scheme), not from the seed
  int64_t mean_rows = 0;            // rows behind the means finalize centred with (centre = 1)
  uint64_t next_ticket = 1;
  hipEvent_t done_ev[kRing] = {};
  hipEvent_t copy_ev[kRing] = {};
  uint64_t ring_ticket[kRing] = {};
  bool ring_host[kRing] = {};
  hipEvent_t slot_consumed[4] = {};
  bool slot_used[4] = {};
  int next_slot = 0;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_free;
  struct Rec { hipEvent_t a, b, c; int kind; };
  std::vector<Rec> recs;
  int64_t prof_n[3] = {0, 0, 0};
  double prof_ms[3] = {0, 0, 0};

  template <typename T> T* at(int64_t off) { return reinterpret_cast<T*>(ws + off); }
  Ctrl* ctrl() { return at<Ctrl>(lay.off_ctrl); }

  sketch_status dev_fail(hipError_t e, const char* what) {
    sticky = SKETCH_E_DEVICE;
    return fail(SKETCH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }
  hipEvent_t take_event() {
    if (!ev_free.empty()) { hipEvent_t e = ev_free.back(); ev_free.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

sketch_status check_handle(sketch_t h) {
  if (!h) return fail(SKETCH_E_INVAL, "handle is NULL");
  // a block the kernels found non-finite is reported by the first call after they ran
  if (h->sticky == SKETCH_OK && h->nf_host && *reinterpret_cast<volatile int*>(h->nf_host) != 0)
    h->sticky = SKETCH_E_NONFINITE;
  if (h->sticky != SKETCH_OK)
    return fail(h->sticky, "handle is in a sticky error state (%d)", (int)h->sticky);
  return SKETCH_OK;
}

sketch_status make_omega_ready(sketch_t h) {
  const Layout& L = h->lay;
  hipError_t e = launch_omega_quantize(h->cfg.compute, h->cfg.n, L.NP, h->cfg.l, L.LP,
                                       h->at<double>(L.off_om64), h->ws + L.off_omc, h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "omega quantize");
  return SKETCH_OK;
}

sketch_status start_pass(sketch_t h) {
  const Layout& L = h->lay;
  hipError_t e = launch_fill_f64(h->at<double>(L.off_H), (int64_t)L.LP * L.NP, 0.0, h->stream);
  if (e == hipSuccess)
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(h->ctrl()), sizeof(Ctrl) / 4, 0u, h->stream);
  if (e == hipSuccess)
    e = launch_fill_u32(h->at<uint32_t>(L.off_cnt), gemm2_strips(h->cfg.n, h->cfg.compute), 0u,
                        h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "reset state");
  h->rows = 0;
  if (h->cfg.omega_from_seed) {
    h->omega_derived = false;
    e = launch_omega_philox(h->cfg.seed, h->cfg.n, h->cfg.l, h->at<double>(L.off_om64), L.NP,
                            h->stream);
    if (e != hipSuccess) return h->dev_fail(e, "omega generation");
    sketch_status st = make_omega_ready(h);
    if (st != SKETCH_OK) return st;
    h->phase = 1;
  } else {
    h->phase = (h->phase == 0) ? 0 : 1;   // a supplied Omega' stays valid across resets
  }
  return SKETCH_OK;
}

// Enqueues the pass kernels of one block (Alg. 4 steps 6-7) of device rows A (lda elements,
// format src_dtype) at row h->rows of G; with `rec`, HIP events around the two products.
hipError_t enqueue_pass(sketch_t h, const void* A, int64_t lda, int src_dtype, int64_t nrows,
                        sketch_s::Rec* rec) {
  const sketch_config& c = h->cfg;
  const Layout& L = h->lay;
  hipError_t e = hipSuccess;
  PassItem it{};
  it.A = A;
  it.lda = lda;
  it.nrows = (int)nrows;
  it.n = c.n;
  it.omc = h->ws + L.off_omc;
  it.NP = L.NP;
  it.P1 = h->ws + L.off_P1;
  it.ldp = L.RBP;
  it.Gop = h->ws + L.off_Gop;
  it.P2 = h->ws + L.off_P2;
  it.counters = h->at<unsigned>(L.off_cnt);
  it.G = h->ws + L.off_G;
  it.ldg = L.MCAP;
  it.g_row0 = h->rows;
  it.H = h->at<double>(L.off_H);
  it.ldh = L.NP;
  it.fp8_exp = nullptr;
  it.ctrl = h->ctrl();
  it.nf_host = h->nf_dev;
  it.sum_col = c.centre ? c.l : 0;
  int src = src_dtype;
  if (c.compute == SKETCH_FP8_E4M3) {
    uint32_t* amax = h->at<uint32_t>(L.off_fp8);
    int* ex = reinterpret_cast<int*>(amax + 4);
    uint8_t* q = h->ws + L.off_fp8q;
    e = launch_fp8_quantize((const float*)A, lda, (int)nrows, c.n, amax, q, L.NQ, ex,
                            &h->ctrl()->nonfinite, h->nf_dev, h->stream);
    if (e != hipSuccess) return e;
    it.A = q;
    it.lda = L.NQ;
    src = SKETCH_FP8_E4M3;
    it.fp8_exp = ex;
  }
  plan_item(it, c.compute, src, L.splits_max);
  PassGroup a{};
  a.mode = c.compute;
  a.src = src;
  a.LP = L.LP;
  a.NT = L.NT;
  plan_group(a, &it, 1);

  if (rec) {
    rec->a = h->take_event(); rec->b = h->take_event(); rec->c = h->take_event(); rec->kind = 0;
    if (!rec->a || !rec->b || !rec->c) return hipErrorOutOfMemory;
    e = hipEventRecord(rec->a, h->stream);
  }
  if (e == hipSuccess) e = launch_gemm1(a, h->stream);
  if (e == hipSuccess) e = launch_reduce1(a, h->stream);
  if (e == hipSuccess && rec) e = hipEventRecord(rec->b, h->stream);
  if (e == hipSuccess) e = launch_gemm2(a, h->stream);
  if (e == hipSuccess && rec) e = hipEventRecord(rec->c, h->stream);
  return e;
}

// Alg. 4 steps 9-19 for a validated handle in the ingesting state; waits for the stream.
sketch_status finalize_core(sketch_t h, double* S_dev, double* U_dev, int64_t ldu, double* V_dev,
                            int64_t ldv, int32_t* rank_out) {
  const sketch_config& c = h->cfg;
  const Layout& L = h->lay;
  hipError_t e = hipSuccess;
  hipEvent_t fa = nullptr, fb = nullptr;
  if (h->prof) {
    fa = h->take_event(); fb = h->take_event();
    e = hipEventRecord(fa, h->stream);
  }
  if (h->rows == 0) {
    if (e == hipSuccess) e = launch_fill_f64(S_dev, c.k, 0.0, h->stream);
    if (e == hipSuccess) e = launch_fill_rows(V_dev, c.n, c.k, ldv, 0.0, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->dev_fail(e, "finalize");
    if (rank_out) *rank_out = 0;
    h->phase = 2;
    return SKETCH_OK;
  }
  FinalizeArgs f{};
  f.mode = c.compute;
  f.m = h->rows;
  f.n = c.n;
  f.k = c.k;
  f.l = c.l;
  f.b = c.b;
  f.LP = L.LP;
  f.G = h->ws + L.off_G;
  f.ldg = L.MCAP;
  f.H = h->at<double>(L.off_H);
  f.ldh = L.NP;
  f.om64 = h->at<double>(L.off_om64);
  f.ldo = L.NP;
  f.Q = h->at<double>(L.off_Q);
  f.ldq = L.MCAP;
  f.Q2 = (c.b == c.l) ? h->at<double>(L.off_Q2) : nullptr;
  f.Bt = h->at<double>(L.off_Bt);
  f.Qb = h->at<double>(L.off_Qb);
  f.ldb = L.NP;
  f.tsqr_ws = h->at<double>(L.off_tsqr);
  f.tsqr_ws_elems = L.tsqr_elems;
  f.red_ws = h->at<double>(L.off_red);
  f.red_ws_elems = L.red_elems;
  f.small = h->at<double>(L.off_small);
  f.ctrl = h->ctrl();
  f.S = S_dev;
  f.U = U_dev;
  f.ldu = ldu;
  f.V = V_dev;
  f.ldv = ldv;
  f.force_loop = h->force_loop;
  f.force_rb = h->force_rb;
  f.centre = c.centre;
  f.mu = c.centre ? h->at<double>(L.off_mu) : nullptr;
  f.host_pin = h->fin_pin;
  f.host_ev = h->fin_ev;
  Ctrl hc;
  f.ctrl_host = &hc;
  if (e == hipSuccess) e = run_finalize(f, h->stream);
  if (e == hipSuccess && h->prof) e = hipEventRecord(fb, h->stream);
  if (e == hipSuccess && !f.ctrl_read)
    e = read_back(&hc, h->ctrl(), sizeof(Ctrl), h->stream, h->fin_pin, h->fin_ev);
  if (e != hipSuccess) return h->dev_fail(e, "finalize");
  if (h->prof) h->recs.push_back({fa, fb, nullptr, 2});
  h->phase = 2;
  h->mean_rows = h->rows;
  h->path_loop = f.path_loop;
  h->path_rb = f.path_rb;
  if (hc.nonfinite) {
    h->sticky = SKETCH_E_NONFINITE;
    return fail(SKETCH_E_NONFINITE, "an ingested block held NaN or Inf");
  }
  if (rank_out) *rank_out = hc.l_eff;
  return SKETCH_OK;
}

bool is_pinned_host(const void* p) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeHost;
}

}  // namespace

extern "C" {

const char* sketch_last_error(void) { return g_err.c_str(); }

size_t sketch_workspace_size(const sketch_config* cfg) {
  if (const char* why = validate(cfg)) {
    fail(SKETCH_E_INVAL, "%s", why);
    return 0;
  }
  return (size_t)plan(cfg).total;
}

sketch_status sketch_init(sketch_t* out, const sketch_config* cfg, void* dev_ws, size_t ws_bytes,
                          void* hip_stream) {
  if (!out) return fail(SKETCH_E_INVAL, "out is NULL");
  *out = nullptr;
  if (const char* why = validate(cfg)) return fail(SKETCH_E_INVAL, "%s", why);
  const Layout L = plan(cfg);
  if (!dev_ws) return fail(SKETCH_E_INVAL, "workspace is NULL");
  if (((uintptr_t)dev_ws) % kAlign) return fail(SKETCH_E_INVAL, "workspace must be 256-byte aligned");
  if ((int64_t)ws_bytes < L.total)
    return fail(SKETCH_E_NOMEM, "workspace holds %zu bytes, %lld needed", ws_bytes,
                (long long)L.total);
  {
    hipError_t e = finalize_prepare();
    if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "kernel attributes: %s", hipGetErrorString(e));
  }
  sketch_s* h = new sketch_s();
  h->cfg = *cfg;
  h->lay = L;
  h->ws = (uint8_t*)dev_ws;
  h->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess && cfg->host_slots > 0)
    e = hipStreamCreateWithFlags(&h->copy, hipStreamNonBlocking);
  for (int i = 0; i < kRing && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&h->done_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->copy_ev[i], hipEventDisableTiming);
  }
  for (int i = 0; i < cfg->host_slots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&h->slot_consumed[i], hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&h->nf_host, 64, hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    *reinterpret_cast<volatile int*>(h->nf_host) = 0;
    e = hipHostGetDevicePointer((void**)&h->nf_dev, h->nf_host, 0);
  }
  if (e == hipSuccess) e = hipHostMalloc(&h->fin_pin, kHostPinBytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fin_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    sketch_destroy(h);
    return fail(SKETCH_E_DEVICE, "stream/event creation: %s", hipGetErrorString(e));
  }
  // the finalize's small matrices start defined (no kernel reads them before writing, but a
  // rejected factorisation must never meet uninitialised memory)
  e = launch_fill_f64(h->at<double>(L.off_small), (int64_t)finalize_small_elems(cfg->l, cfg->b),
                      0.0, h->stream);
  if (e != hipSuccess) {
    sketch_destroy(h);
    return fail(SKETCH_E_DEVICE, "workspace clear: %s", hipGetErrorString(e));
  }
  sketch_status st = start_pass(h);
  if (st != SKETCH_OK) {
    sketch_destroy(h);
    return st;
  }
  *out = h;
  return SKETCH_OK;
}

sketch_status sketch_reset(sketch_t h, uint64_t seed) {
  if (sketch_status st = check_handle(h)) return st;
  h->cfg.seed = seed;
  return start_pass(h);
}

sketch_status sketch_set_omega(sketch_t h, const double* omega_dev, int64_t ld) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->cfg.omega_from_seed) return fail(SKETCH_E_STATE, "handle draws its own Omega");
  if (h->rows > 0 || h->phase == 2) return fail(SKETCH_E_STATE, "Omega must precede the first ingest");
  if (!omega_dev || ld < h->cfg.l) return fail(SKETCH_E_INVAL, "bad Omega pointer or ld");
  const Layout& L = h->lay;
  hipError_t e = launch_fill_f64(h->at<double>(L.off_om64), (int64_t)L.LP * L.NP, 0.0, h->stream);
  if (e == hipSuccess)
    e = launch_omega_user(omega_dev, ld, h->cfg.n, h->cfg.l, h->at<double>(L.off_om64), L.NP,
                          h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "set omega");
  sketch_status st = make_omega_ready(h);
  if (st != SKETCH_OK) return st;
  h->phase = 1;
  return SKETCH_OK;
}

sketch_status sketch_ingest_block(sketch_t h, const void* rows, int32_t src_dtype, int64_t nrows,
                                  int64_t ld, int32_t src_is_device, uint64_t* ticket) {
  if (sketch_status st = check_handle(h)) return st;
  const sketch_config& c = h->cfg;
  const Layout& L = h->lay;
  if (h->phase == 0) return fail(SKETCH_E_STATE, "Omega has not been supplied");
  if (h->phase == 2) return fail(SKETCH_E_STATE, "ingest after finalize (call sketch_reset)");
  if (!rows) return fail(SKETCH_E_INVAL, "rows is NULL");
  if (nrows < 1) return fail(SKETCH_E_INVAL, "nrows must be >= 1");
  if (ld < c.n) return fail(SKETCH_E_INVAL, "ld must be >= n");
  if (src_is_device != 0 && src_is_device != 1) return fail(SKETCH_E_INVAL, "src_is_device must be 0 or 1");
  if (!mode_accepts(c.compute, src_dtype))
    return fail(SKETCH_E_INVAL, "source format %d not supported by compute mode %d", src_dtype,
                c.compute);
  if (nrows > c.max_block_rows)
    return fail(SKETCH_E_CAPACITY, "block of %lld rows exceeds max_block_rows %lld",
                (long long)nrows, (long long)c.max_block_rows);
  if (h->rows + nrows > c.m_capacity)
    return fail(SKETCH_E_CAPACITY, "m_capacity %lld exceeded", (long long)c.m_capacity);
  const int es = src_size(src_dtype);
  const void* A = rows;
  int64_t lda = ld;
  const uint64_t tk = h->next_ticket;
  const int ring = (int)(tk % kRing);
  hipError_t e = hipSuccess;
  int slot = -1;
  if (!src_is_device) {
    if (c.host_slots == 0) return fail(SKETCH_E_INVAL, "handle has no host staging slots");
    if (src_dtype != c.host_src) return fail(SKETCH_E_INVAL, "src_dtype differs from host_src");
    if (!is_pinned_host(rows)) return fail(SKETCH_E_INVAL, "host rows must be pinned (hipHostMalloc)");
    slot = h->next_slot;
    h->next_slot = (h->next_slot + 1) % c.host_slots;
    uint8_t* dst = h->ws + L.off_stage + (int64_t)slot * L.stage_slot_bytes;
    if (h->slot_used[slot]) e = hipStreamWaitEvent(h->copy, h->slot_consumed[slot], 0);
    // contiguous rows whose length keeps 16-byte alignment go as one linear copy; others as a
    // pitched copy into rows padded to 64 elements
    const bool linear = (ld == c.n) && ((c.n * es) % 16 == 0);
    if (e == hipSuccess) {
      if (linear)
        e = hipMemcpyAsync(dst, rows, (size_t)(nrows * c.n * es), hipMemcpyHostToDevice, h->copy);
      else
        e = hipMemcpy2DAsync(dst, L.LDST * es, rows, ld * es, c.n * es, nrows,
                             hipMemcpyHostToDevice, h->copy);
    }
    lda = linear ? c.n : L.LDST;
    if (e == hipSuccess) e = hipEventRecord(h->copy_ev[ring], h->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->copy_ev[ring], 0);
    if (e != hipSuccess) return h->dev_fail(e, "host block copy");
    A = dst;
  }

  sketch_s::Rec rec{};
  if (e == hipSuccess) e = enqueue_pass(h, A, lda, src_dtype, nrows, h->prof ? &rec : nullptr);
  if (e == hipErrorOutOfMemory) return h->dev_fail(e, "profiling events");
  if (e == hipSuccess) e = hipEventRecord(h->done_ev[ring], h->stream);
  if (e == hipSuccess && slot >= 0) {
    e = hipEventRecord(h->slot_consumed[slot], h->stream);
    h->slot_used[slot] = true;
  }
  if (e != hipSuccess) return h->dev_fail(e, "pass kernels");
  if (h->prof) h->recs.push_back(rec);
  h->ring_ticket[ring] = tk;
  h->ring_host[ring] = (slot >= 0);
  h->next_ticket = tk + 1;
  h->rows += nrows;
  if (ticket) *ticket = tk;
  return SKETCH_OK;
}

sketch_status sketch_poll(sketch_t h, uint64_t ticket, int32_t* done) {
  if (sketch_status st = check_handle(h)) return st;
  if (!done) return fail(SKETCH_E_INVAL, "done is NULL");
  if (ticket == 0 || ticket >= h->next_ticket) return fail(SKETCH_E_INVAL, "unknown ticket");
  const int ring = (int)(ticket % kRing);
  hipEvent_t ev;
  if (h->ring_ticket[ring] == ticket)
    ev = h->ring_host[ring] ? h->copy_ev[ring] : h->done_ev[ring];
  else
    ev = h->done_ev[ring];   // a later ticket reused the slot; its completion implies ours
  hipError_t e = hipEventQuery(ev);
  if (e == hipSuccess) { *done = 1; return SKETCH_OK; }
  if (e == hipErrorNotReady) { *done = 0; return SKETCH_OK; }
  return h->dev_fail(e, "poll");
}

sketch_status sketch_finalize(sketch_t h, double* S_dev, double* U_dev, int64_t ldu,
                              double* V_dev, int64_t ldv, int32_t* rank_out) {
  if (sketch_status st = check_handle(h)) return st;
  const sketch_config& c = h->cfg;
  if (h->phase != 1) return fail(SKETCH_E_STATE, h->phase == 2 ? "already finalized" : "Omega has not been supplied");
  if (!S_dev || !V_dev) return fail(SKETCH_E_INVAL, "S and V are required");
  if (ldv < c.k) return fail(SKETCH_E_INVAL, "ldv must be >= k");
  if (U_dev && !c.want_u) return fail(SKETCH_E_INVAL, "U requested but want_u = 0");
  if (U_dev && ldu < c.k) return fail(SKETCH_E_INVAL, "ldu must be >= k");
  return finalize_core(h, S_dev, U_dev, ldu, V_dev, ldv, rank_out);
}

sketch_status sketch_power_restart(sketch_t h, int32_t route, int32_t* route_used) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase != 1 || h->rows == 0)
    return fail(SKETCH_E_STATE, "the power scheme needs a completed first pass (rows ingested, "
                                "not finalized)");
  if (route != 0 && route != 1 && route != 2) return fail(SKETCH_E_INVAL, "route must be 0, 1 or 2");
  const Layout& L = h->lay;
  PowerArgs p{};
  p.n = h->cfg.n;
  p.l = h->cfg.l;
  p.b = h->cfg.b;
  p.H = h->at<double>(L.off_H);
  p.ldh = L.NP;
  p.om64 = h->at<double>(L.off_om64);
  p.ldo = L.NP;
  p.W1 = h->at<double>(L.off_Bt);
  p.W2 = h->at<double>(L.off_Qb);
  p.ldw = L.NP;
  p.red_ws = h->at<double>(L.off_red);
  p.tsqr_ws = h->at<double>(L.off_tsqr);
  p.small = h->at<double>(L.off_small);
  p.route = route;
  p.host_pin = h->fin_pin;
  p.host_ev = h->fin_ev;
  hipError_t e = hipSuccess;
  if (h->cfg.centre)   // Omega_2 from the centred sketch: orth(A_c^T A_c Omega)
    e = centre_sketch(h->cfg.compute, h->ws + L.off_G, L.MCAP, h->rows, h->at<double>(L.off_H),
                      L.NP, h->cfg.n, h->cfg.l, h->at<double>(L.off_om64), L.NP,
                      h->at<double>(L.off_mu), h->at<double>(L.off_small), h->cfg.b, h->stream);
  if (e == hipSuccess) e = run_power_omega(p, h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "power scheme: orth(H)");
  // Omega_2 rounded to the operand format, then a fresh pass with it
  if (sketch_status st = make_omega_ready(h)) return st;
  const int seed_flag = h->cfg.omega_from_seed;
  h->cfg.omega_from_seed = 0;
  sketch_status st = start_pass(h);
  h->cfg.omega_from_seed = seed_flag;
  if (st != SKETCH_OK) return st;
  e = read_back(nullptr, nullptr, 0, h->stream, h->fin_pin, h->fin_ev);
  if (e != hipSuccess) return h->dev_fail(e, "power scheme");
  h->omega_derived = true;
  h->phase = 1;
  if (route_used) *route_used = p.route_used;
  return SKETCH_OK;
}

sketch_status sketch_column_mean(sketch_t h, double* mu_dev) {
  if (sketch_status st = check_handle(h)) return st;
  if (!h->cfg.centre) return fail(SKETCH_E_STATE, "the handle does not centre (centre = 0)");
  if (!mu_dev) return fail(SKETCH_E_INVAL, "mu is NULL");
  const Layout& L = h->lay;
  hipError_t e;
  if (h->phase == 2) {
    if (h->mean_rows == 0) return fail(SKETCH_E_STATE, "no rows were ingested");
    e = hipMemcpyAsync(mu_dev, h->at<double>(L.off_mu), h->cfg.n * 8, hipMemcpyDeviceToDevice,
                       h->stream);
  } else {
    if (h->rows == 0) return fail(SKETCH_E_STATE, "no rows were ingested");
    e = hipMemcpyAsync(mu_dev, h->at<double>(L.off_H) + (int64_t)h->cfg.l * L.NP, h->cfg.n * 8,
                       hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = launch_scale_f64(mu_dev, h->cfg.n, 1.0 / (double)h->rows, h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "column mean");
  return SKETCH_OK;
}

sketch_status sketch_debug_force_paths(sketch_t h, int32_t loop_householder, int32_t rb_mode) {
  if (sketch_status st = check_handle(h)) return st;
  if (rb_mode < 0 || rb_mode > 4) return fail(SKETCH_E_INVAL, "rb mode must be 0 .. 4");
  h->force_loop = loop_householder ? 1 : 0;
  h->force_rb = rb_mode;
  return SKETCH_OK;
}

sketch_status sketch_finalize_paths(sketch_t h, int32_t* loop_path, int32_t* rb_path) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase != 2) return fail(SKETCH_E_STATE, "not finalized");
  if (loop_path) *loop_path = h->path_loop;
  if (rb_path) *rb_path = h->path_rb;
  return SKETCH_OK;
}

sketch_status sketch_get_omega(sketch_t h, double* omega_dev, int64_t ld) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase == 0) return fail(SKETCH_E_STATE, "Omega has not been supplied");
  if (!omega_dev || ld < h->cfg.l) return fail(SKETCH_E_INVAL, "bad output pointer or ld");
  hipError_t e = launch_copy_omega_out(h->at<double>(h->lay.off_om64), h->lay.NP, h->cfg.n,
                                       h->cfg.l, omega_dev, ld, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "get omega");
  return SKETCH_OK;
}

sketch_status sketch_debug_state(sketch_t h, double* G_dev, double* H_dev, int64_t* rows_out) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase == 2) return fail(SKETCH_E_STATE, "state is consumed by finalize");
  hipError_t e = launch_copy_state(h->cfg.compute, h->ws + h->lay.off_G, h->lay.MCAP, h->rows,
                                   h->at<double>(h->lay.off_H), h->lay.NP, h->cfg.n, h->cfg.l,
                                   G_dev, H_dev, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "debug state");
  if (rows_out) *rows_out = h->rows;
  return SKETCH_OK;
}

// ---------------------------------------------------------------- checkpoint, restore, merge
}  // extern "C"

namespace {

constexpr uint64_t kCkptMagic = 0x314b43414350534bull;   // "KSPCACK1" little-endian
constexpr uint32_t kCkptVersion = 1;

// Layout of a checkpoint in host memory: this header, then H (hcols columns of n FP64 values),
// then G (l columns of `rows` values of g_bytes each), then Omega' (l columns of n FP64 values)
// when it was supplied rather than drawn from the seed.  Every section starts 64-byte aligned.
struct CkptHeader {
  uint64_t magic;
  uint32_t version, header_bytes;
  int64_t n, rows;
  int32_t l, compute, omega_from_seed, g_bytes;
  int32_t hcols, centre;
  uint64_t seed;
  int64_t off_H, off_G, off_om, total;
  int64_t pad1[4];
};

CkptHeader ckpt_header(const sketch_s* h) {
  CkptHeader c;
  memset(&c, 0, sizeof(c));
  c.magic = kCkptMagic;
  c.version = kCkptVersion;
  c.header_bytes = sizeof(CkptHeader);
  c.n = h->cfg.n;
  c.rows = h->rows;
  c.l = h->cfg.l;
  c.compute = h->cfg.compute;
  c.omega_from_seed = (h->cfg.omega_from_seed && !h->omega_derived) ? 1 : 0;
  c.g_bytes = (h->cfg.compute == SKETCH_F64) ? 8 : 4;
  c.hcols = h->cfg.l + (h->cfg.centre ? 1 : 0);   // with centring, column l holds A^T 1
  c.centre = h->cfg.centre;
  c.seed = h->cfg.seed;
  int64_t off = rup<int64_t>(sizeof(CkptHeader), 64);
  c.off_H = off;
  off += rup<int64_t>((int64_t)c.hcols * c.n * 8, 64);
  c.off_G = off;
  off += rup<int64_t>((int64_t)c.l * c.rows * c.g_bytes, 64);
  c.off_om = c.omega_from_seed ? 0 : off;
  if (!c.omega_from_seed) off += rup<int64_t>((int64_t)c.l * c.n * 8, 64);
  c.total = off;
  return c;
}

// Checks a checkpoint against the handle it is read into; returns the header through *out.
sketch_status ckpt_check(sketch_t h, const void* buf, size_t bytes, CkptHeader* out) {
  if (!buf) return fail(SKETCH_E_INVAL, "checkpoint buffer is NULL");
  if (bytes < sizeof(CkptHeader)) return fail(SKETCH_E_INVAL, "checkpoint buffer too small");
  CkptHeader c;
  memcpy(&c, buf, sizeof(c));
  if (c.magic != kCkptMagic || c.version != kCkptVersion || c.header_bytes != sizeof(CkptHeader))
    return fail(SKETCH_E_INVAL, "not a checkpoint of this library version");
  if (c.n != h->cfg.n || c.l != h->cfg.l || c.compute != h->cfg.compute ||
      c.centre != h->cfg.centre)
    return fail(SKETCH_E_INVAL,
                "checkpoint of n=%lld l=%d compute=%d centre=%d does not fit this handle",
                (long long)c.n, c.l, c.compute, c.centre);
  if (c.rows < 0 || c.hcols != c.l + c.centre ||
      c.g_bytes != ((c.compute == SKETCH_F64) ? 8 : 4))
    return fail(SKETCH_E_INVAL, "corrupt checkpoint header");
  // recompute the section offsets from the header's own sizes
  sketch_s tmp;
  tmp.cfg = h->cfg;
  tmp.cfg.omega_from_seed = c.omega_from_seed;
  tmp.cfg.seed = c.seed;
  tmp.omega_derived = false;
  tmp.rows = c.rows;
  const CkptHeader e = ckpt_header(&tmp);
  if (e.off_H != c.off_H || e.off_G != c.off_G || e.off_om != c.off_om || e.total != c.total)
    return fail(SKETCH_E_INVAL, "corrupt checkpoint header");
  if ((int64_t)bytes < c.total) return fail(SKETCH_E_INVAL, "checkpoint truncated");
  *out = c;
  return SKETCH_OK;
}

// Writes the checkpoint's Omega' (FP64, column-major, ld NP) to `dst` on the handle's stream; a
// seed-drawn one is drawn and rounded again, its operand copy going to `omc_dst`.  A supplied one
// is stored already rounded and is copied as it is.
hipError_t ckpt_omega(sketch_t h, const CkptHeader& c, const uint8_t* buf, double* dst,
                      void* omc_dst) {
  const Layout& L = h->lay;
  hipError_t e = launch_fill_f64(dst, (int64_t)L.LP * L.NP, 0.0, h->stream);
  if (e != hipSuccess) return e;
  if (c.omega_from_seed) {
    e = launch_omega_philox(c.seed, c.n, c.l, dst, L.NP, h->stream);
    if (e == hipSuccess)
      e = launch_omega_quantize(h->cfg.compute, c.n, L.NP, c.l, L.LP, dst, omc_dst, h->stream);
    return e;
  }
  return hipMemcpy2DAsync(dst, L.NP * 8, buf + c.off_om, c.n * 8, c.n * 8, c.l,
                          hipMemcpyHostToDevice, h->stream);
}

}  // namespace

extern "C" {

size_t sketch_checkpoint_size(sketch_t h) {
  if (check_handle(h) != SKETCH_OK) return 0;
  if (h->phase != 1) {
    fail(SKETCH_E_STATE, "no pass state to checkpoint");
    return 0;
  }
  return (size_t)ckpt_header(h).total;
}

sketch_status sketch_checkpoint(sketch_t h, void* buf, size_t bytes) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase != 1) return fail(SKETCH_E_STATE, "no pass state to checkpoint");
  if (!buf) return fail(SKETCH_E_INVAL, "checkpoint buffer is NULL");
  const CkptHeader c = ckpt_header(h);
  if ((int64_t)bytes < c.total)
    return fail(SKETCH_E_INVAL, "checkpoint needs %lld bytes", (long long)c.total);
  const Layout& L = h->lay;
  uint8_t* out = (uint8_t*)buf;
  memcpy(out, &c, sizeof(c));
  hipError_t e = hipMemcpy2DAsync(out + c.off_H, c.n * 8, h->at<double>(L.off_H), L.NP * 8,
                                  c.n * 8, c.hcols, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && c.rows > 0)
    e = hipMemcpy2DAsync(out + c.off_G, c.rows * c.g_bytes, h->ws + L.off_G, L.MCAP * c.g_bytes,
                         c.rows * c.g_bytes, c.l, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && !c.omega_from_seed)
    e = hipMemcpy2DAsync(out + c.off_om, c.n * 8, h->at<double>(L.off_om64), L.NP * 8, c.n * 8,
                         c.l, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "checkpoint");
  // a block the kernels found non-finite must not be saved as a valid state
  if (*reinterpret_cast<volatile int*>(h->nf_host) != 0) {
    h->sticky = SKETCH_E_NONFINITE;
    return fail(SKETCH_E_NONFINITE, "an ingested block held NaN or Inf");
  }
  return SKETCH_OK;
}

sketch_status sketch_restore(sketch_t h, const void* buf, size_t bytes) {
  if (sketch_status st = check_handle(h)) return st;
  CkptHeader c;
  if (sketch_status st = ckpt_check(h, buf, bytes, &c)) return st;
  if (c.rows > h->cfg.m_capacity)
    return fail(SKETCH_E_CAPACITY, "checkpoint holds %lld rows, m_capacity is %lld",
                (long long)c.rows, (long long)h->cfg.m_capacity);
  const Layout& L = h->lay;
  const uint8_t* in = (const uint8_t*)buf;
  // a fresh pass (H = 0, counters and flags cleared), then the checkpoint's state over it
  const int saved_seed_flag = h->cfg.omega_from_seed;
  h->cfg.omega_from_seed = 0;            // start_pass must not draw an Omega of its own
  sketch_status st = start_pass(h);
  h->cfg.omega_from_seed = saved_seed_flag;
  if (st != SKETCH_OK) return st;
  hipError_t e = ckpt_omega(h, c, in, h->at<double>(L.off_om64), h->ws + L.off_omc);
  if (e == hipSuccess && !c.omega_from_seed)
    e = launch_omega_quantize(h->cfg.compute, c.n, L.NP, c.l, L.LP, h->at<double>(L.off_om64),
                              h->ws + L.off_omc, h->stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(h->at<double>(L.off_H), L.NP * 8, in + c.off_H, c.n * 8, c.n * 8, c.hcols,
                         hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && c.rows > 0)
    e = hipMemcpy2DAsync(h->ws + L.off_G, L.MCAP * c.g_bytes, in + c.off_G, c.rows * c.g_bytes,
                         c.rows * c.g_bytes, c.l, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "restore");
  h->cfg.seed = c.seed;
  h->omega_derived = !c.omega_from_seed && h->cfg.omega_from_seed;
  h->rows = c.rows;
  h->phase = 1;
  return SKETCH_OK;
}

sketch_status sketch_merge(sketch_t h, const void* buf, size_t bytes) {
  if (sketch_status st = check_handle(h)) return st;
  if (h->phase != 1) return fail(SKETCH_E_STATE, "merge needs a handle that is ingesting");
  CkptHeader c;
  if (sketch_status st = ckpt_check(h, buf, bytes, &c)) return st;
  if (h->rows + c.rows > h->cfg.m_capacity)
    return fail(SKETCH_E_CAPACITY, "merged rows exceed m_capacity %lld",
                (long long)h->cfg.m_capacity);
  const Layout& L = h->lay;
  const uint8_t* in = (const uint8_t*)buf;
  double* tmp = h->at<double>(L.off_Bt);             // n-side scratch of the finalize
  unsigned* diff = reinterpret_cast<unsigned*>(h->ws + L.off_fp8 + 32);
  unsigned ndiff = 0;
  // the two sketches must come from the same Omega' (Eq. 10 sums A_i^T A_i Omega)
  hipError_t e = launch_fill_u32(diff, 1, 0u, h->stream);
  if (e == hipSuccess) e = ckpt_omega(h, c, in, tmp, h->ws + L.off_Qb);
  if (e == hipSuccess)
    e = launch_count_diff(tmp, L.NP, h->at<double>(L.off_om64), L.NP, c.n, c.l, diff, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&ndiff, diff, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "merge");
  if (ndiff != 0) return fail(SKETCH_E_INVAL, "checkpoint was taken with a different Omega");
  // H = H + H', G = [G; G']
  e = hipMemcpy2DAsync(tmp, L.NP * 8, in + c.off_H, c.n * 8, c.n * 8, c.hcols,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = launch_add_cols(h->at<double>(L.off_H), L.NP, tmp, L.NP, c.n, c.hcols, h->stream);
  if (e == hipSuccess && c.rows > 0)
    e = hipMemcpy2DAsync(h->ws + L.off_G + h->rows * c.g_bytes, L.MCAP * c.g_bytes, in + c.off_G,
                         c.rows * c.g_bytes, c.rows * c.g_bytes, c.l, hipMemcpyHostToDevice,
                         h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "merge");
  h->rows += c.rows;
  return SKETCH_OK;
}

sketch_status sketch_philox_words(uint64_t seed, uint64_t first, int64_t count, uint64_t* out_dev,
                                  void* hip_stream) {
  if (count < 0 || (count > 0 && !out_dev)) return fail(SKETCH_E_INVAL, "bad output");
  if (count == 0) return SKETCH_OK;
  hipError_t e = launch_philox_words(seed, first, count, out_dev, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "philox: %s", hipGetErrorString(e));
  return SKETCH_OK;
}

sketch_status sketch_jacobi_schedule(int32_t n, uint8_t* pairs, int64_t capacity,
                                     int32_t* rounds) {
  if (!rounds) return fail(SKETCH_E_INVAL, "bad arguments");
  const int r = jacobi_schedule(n, pairs, capacity);
  if (r < 0) return fail(SKETCH_E_INVAL, "n outside 0..128 or the table does not fit");
  *rounds = r;
  return SKETCH_OK;
}

sketch_status sketch_profile_enable(sketch_t h, int32_t on) {
  if (sketch_status st = check_handle(h)) return st;
  h->prof = (on != 0);
  return SKETCH_OK;
}

sketch_status sketch_profile_read(sketch_t h, int32_t kind, int64_t* launches, double* total_ms) {
  if (sketch_status st = check_handle(h)) return st;
  if (kind < 0 || kind > 2 || !launches || !total_ms) return fail(SKETCH_E_INVAL, "bad arguments");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->dev_fail(e, "profile sync");
  for (auto& r : h->recs) {
    float ms = 0.f;
    if (r.kind == 0) {
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) { h->prof_ms[0] += ms; h->prof_n[0]++; }
      if (hipEventElapsedTime(&ms, r.b, r.c) == hipSuccess) { h->prof_ms[1] += ms; h->prof_n[1]++; }
      h->ev_free.push_back(r.c);
    } else {
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) { h->prof_ms[2] += ms; h->prof_n[2]++; }
    }
    h->ev_free.push_back(r.a);
    h->ev_free.push_back(r.b);
  }
  h->recs.clear();
  *launches = h->prof_n[kind];
  *total_ms = h->prof_ms[kind];
  h->prof_n[kind] = 0;
  h->prof_ms[kind] = 0.0;
  return SKETCH_OK;
}

sketch_status sketch_destroy(sketch_t h) {
  if (!h) return fail(SKETCH_E_INVAL, "handle is NULL");
  (void)hipStreamSynchronize(h->stream);
  if (h->copy) { (void)hipStreamSynchronize(h->copy); (void)hipStreamDestroy(h->copy); }
  for (int i = 0; i < kRing; ++i) {
    if (h->done_ev[i]) (void)hipEventDestroy(h->done_ev[i]);
    if (h->copy_ev[i]) (void)hipEventDestroy(h->copy_ev[i]);
  }
  for (int i = 0; i < 4; ++i)
    if (h->slot_consumed[i]) (void)hipEventDestroy(h->slot_consumed[i]);
  for (auto& r : h->recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
    if (r.c) (void)hipEventDestroy(r.c);
  }
  for (auto ev : h->ev_free) (void)hipEventDestroy(ev);
  if (h->nf_host) (void)hipHostFree(h->nf_host);
  if (h->fin_pin) (void)hipHostFree(h->fin_pin);
  if (h->fin_ev) (void)hipEventDestroy(h->fin_ev);
  delete h;
  return SKETCH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- single call, no allocation
// The workspace of sketch_pca_static lives in this file-scope device array instead of caller
// memory.  In host code `scratch` only names the symbol: its device address (one per GPU, each
// GPU holding its own copy) comes from hipGetSymbolAddress, taken once per device with that
// device current and kept in g_scratch_dev.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t static_scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

bool is_device_memory(const void* p) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}
}  // namespace

extern "C" {

sketch_status sketch_pca_static(const sketch_config* cfg, const void* A_dev, int32_t src_dtype,
                                int64_t m, int64_t lda, double* S_dev, double* U_dev,
                                int64_t ldu, double* V_dev, int64_t ldv, int32_t* rank_out,
                                void* hip_stream) {
  if (const char* why = validate(cfg)) return fail(SKETCH_E_INVAL, "%s", why);
  if (cfg->host_slots != 0) return fail(SKETCH_E_INVAL, "host_slots must be 0 (device rows only)");
  if (!cfg->omega_from_seed) return fail(SKETCH_E_INVAL, "omega_from_seed must be 1");
  if (!A_dev || !S_dev || !V_dev) return fail(SKETCH_E_INVAL, "A, S and V are required");
  if (m < 1) return fail(SKETCH_E_INVAL, "m must be >= 1");
  if (m > cfg->m_capacity)
    return fail(SKETCH_E_CAPACITY, "m = %lld exceeds m_capacity %lld", (long long)m,
                (long long)cfg->m_capacity);
  if (lda < cfg->n) return fail(SKETCH_E_INVAL, "lda must be >= n");
  if (ldv < cfg->k) return fail(SKETCH_E_INVAL, "ldv must be >= k");
  if (U_dev && (!cfg->want_u || ldu < cfg->k))
    return fail(SKETCH_E_INVAL, "U needs want_u = 1 and ldu >= k");
  if (!mode_accepts(cfg->compute, src_dtype))
    return fail(SKETCH_E_INVAL, "source format %d not supported by compute mode %d", src_dtype,
                cfg->compute);
  if (!is_device_memory(A_dev)) return fail(SKETCH_E_INVAL, "A must be device memory");
  const Layout L = plan(cfg);
  if ((size_t)L.total > kStaticScratchBytes)
    return fail(SKETCH_E_CAPACITY,
                "this configuration needs %lld bytes of workspace; the static scratch holds %zu",
                (long long)L.total, kStaticScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SKETCH_E_DEVICE, "device %d out of range", dev);
  void* ws = nullptr;
  e = static_scratch_address(dev, &ws);
  if (e != hipSuccess)
    return fail(SKETCH_E_DEVICE, "static scratch address: %s", hipGetErrorString(e));
  e = finalize_prepare();
  if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "kernel attributes: %s", hipGetErrorString(e));
  // a handle on the stack over the static scratch: no events, no side stream, no mapped flag
  // (a non-finite block is reported from the device control block at the end)
  sketch_s h;
  h.cfg = *cfg;
  h.lay = L;
  h.ws = (uint8_t*)ws;
  h.stream = (hipStream_t)hip_stream;
  h.device = dev;
  // the scratch keeps the last call's contents: everything read before it is written is cleared
  e = launch_fill_f64(h.at<double>(L.off_small), (int64_t)finalize_small_elems(cfg->l, cfg->b),
                      0.0, h.stream);
  if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "scratch clear: %s", hipGetErrorString(e));
  if (sketch_status st = start_pass(&h)) return st;
  const int es = src_size(src_dtype);
  const uint8_t* A = (const uint8_t*)A_dev;
  for (int64_t r0 = 0; r0 < m; r0 += cfg->max_block_rows) {
    const int64_t rows = std::min<int64_t>(cfg->max_block_rows, m - r0);
    e = enqueue_pass(&h, A + r0 * lda * es, lda, src_dtype, rows, nullptr);
    if (e != hipSuccess) return fail(SKETCH_E_DEVICE, "pass kernels: %s", hipGetErrorString(e));
    h.rows += rows;
  }
  return finalize_core(&h, S_dev, U_dev, ldu, V_dev, ldv, rank_out);
}

}  // extern "C"

