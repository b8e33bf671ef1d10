// Host side of the C ABI: contexts, argument checks, scratch, launches and
// the HIP-graph cache of the batched launch sequence.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "sccg_common.h"

using namespace sccg;

struct sccg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  sccg_params p{};
  std::string msg;
  int cu_count = 1;
  // per-polygon scratch
  Meta* metaA = nullptr;
  int64_t* areaA = nullptr;
  int32_t* bigA = nullptr;
  int64_t capA = 0;
  Meta* metaB = nullptr;
  int64_t* areaB = nullptr;
  int32_t* bigB = nullptr;
  int64_t capB = 0;
  int32_t* big_count = nullptr;  // [2]
  uint32_t* err = nullptr;
  // per-pair scratch
  uint8_t* cls = nullptr;
  PairRec* rec = nullptr;
  int32_t* l_list = nullptr;
  Meta* hbox = nullptr;
  int64_t cap_pairs = 0;
  // batched state and queues
  BatchState* st = nullptr;
  unsigned long long* queue = nullptr;
  int64_t queue_slots = 0;  // allocated n_queues * queue_cap
  int32_t queue_nq = 0, queue_per = 0;  // the layout the queue slots were last cleared for
  unsigned long long* plain_stats = nullptr;
  int stats_on = 0;
  int stamps_on = 0;
  // per-wave stamps of the batched kernels (calls with work counters on)
  unsigned long long* wave_t = nullptr;
  int64_t wave_cap = 0;                        // waves per kernel the buffer holds
  int64_t wave_n[kStampedKernels] = {0, 0, 0};  // waves of each kernel in the last stamped call
  uint32_t last_mode = 0;
  // graph cache for the batched sequence
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  int64_t graph_launches = 0;  // batched calls that ran as a replay of the captured graph
  // filter-stage scratch
  int4* j_bbox = nullptr;
  int4* j_grid = nullptr;
  int64_t* j_cells = nullptr;
  int64_t* j_cell_base = nullptr;
  int64_t* j_sums = nullptr;
  int32_t* j_count = nullptr;
  int64_t* j_start = nullptr;
  int32_t* j_list = nullptr;
  int32_t* j_bcount = nullptr;
  int64_t* j_bstart = nullptr;
  JacAcc* j_acc = nullptr;  // per-set accumulators of sccg_jaccard_sets
  int64_t j_cap[10] = {};
  // kernel timing
  int timing_on = 0;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t ev_used = 0;          // pairs recorded since the last read
};

namespace {

const char* kVersion = "sccg 0.1 (gfx950)";

int fail(sccg_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->msg = buf;
  }
  return code;
}

int hip_fail(sccg_ctx* c, hipError_t e, const char* what) {
  return fail(c, SCCG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                             \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
  } while (0)

int resolve_params(sccg_ctx* c, const sccg_params* in, sccg_params* out) {
  sccg_params p{};
  if (in) p = *in;
  if (p.wg_size == 0) p.wg_size = 64;
  if (p.wg_size != 64 && p.wg_size != 128 && p.wg_size != 256)
    return fail(c, SCCG_E_ARG, "wg_size must be 64, 128 or 256 (got %d)", p.wg_size);
  if (p.split_gx == 0 && p.split_gy == 0) {
    p.split_gx = p.wg_size == 64 ? 8 : 16;
    p.split_gy = p.wg_size / p.split_gx;
  }
  if (p.split_gx * p.split_gy != p.wg_size || p.split_gx < 4 || p.split_gy < 4)
    return fail(c, SCCG_E_ARG, "split grid %dx%d must multiply to wg_size %d with both sides >= 4", p.split_gx,
                p.split_gy, p.wg_size);
  if (p.box_threshold == 0) p.box_threshold = p.wg_size * p.wg_size / 2;
  if (p.box_threshold < 2 || p.box_threshold > (1 << 30))
    return fail(c, SCCG_E_ARG, "box_threshold %d outside [2, 2^30]", p.box_threshold);
  if (p.queue_chunk == 0) p.queue_chunk = 16;
  if (p.queue_chunk < 1 || p.queue_chunk > 64) return fail(c, SCCG_E_ARG, "queue_chunk outside [1, 64]");
  if (p.lds_vertex_cap == 0) p.lds_vertex_cap = 1024;
  if (p.lds_vertex_cap < 1 || p.lds_vertex_cap > 4096)
    return fail(c, SCCG_E_ARG, "lds_vertex_cap outside [1, 4096]");
  const uint32_t known = SCCG_F_NO_LPT | SCCG_F_NO_KNOWN_INSIDE | SCCG_F_NO_SPLIT_QUEUE | SCCG_F_NO_GRAPH |
                         SCCG_F_PIXEL_ONLY | SCCG_F_NO_SEP | SCCG_F_NO_UNION_TILE;
  if (p.flags & ~known) return fail(c, SCCG_E_ARG, "unknown flag bits 0x%x", p.flags & ~known);
  if (p.grid < 0 || p.grid > (1 << 20)) return fail(c, SCCG_E_ARG, "grid outside [0, 2^20]");
  if (p.queue_cap == 0) p.queue_cap = 1 << 20;
  if (p.queue_cap < 1 || p.queue_cap > (1 << 26)) return fail(c, SCCG_E_ARG, "queue_cap outside [1, 2^26]");
  if (p.waves_per_wg == 0) p.waves_per_wg = 4;
  if (p.waves_per_wg < 1 || p.waves_per_wg > 8) return fail(c, SCCG_E_ARG, "waves_per_wg outside [1, 8]");
  if (p.min_queue_cells == 0) p.min_queue_cells = 8;
  if (p.min_queue_cells < 1 || p.min_queue_cells > 65) return fail(c, SCCG_E_ARG, "min_queue_cells outside [1, 65]");
  if (p.n_queues == 0) p.n_queues = kMaxGrid;
  if (p.n_queues < 1 || p.n_queues > kMaxGrid) return fail(c, SCCG_E_ARG, "n_queues outside [1, 8]");
  if (p.heavy_verts == 0) p.heavy_verts = 512;
  if (p.heavy_verts < 1) return fail(c, SCCG_E_ARG, "heavy_verts < 1");
  if (p.min_classify_cells == 0) p.min_classify_cells = 26;
  if (p.min_classify_cells < 1 || p.min_classify_cells > 65)
    return fail(c, SCCG_E_ARG, "min_classify_cells outside [1, 65]");
  if (p.sweep_pair_box == 0) p.sweep_pair_box = 1;
  if (p.sweep_pair_box < 1 || p.sweep_pair_box > 2) return fail(c, SCCG_E_ARG, "sweep_pair_box must be 1 or 2");
  *out = p;
  return SCCG_OK;
}

// The captured graph holds the scratch pointers as kernel arguments: it is
// dropped whenever scratch it may use is freed or reallocated.
void drop_graph(sccg_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gkey.clear();
}

template <typename T>
int grow(sccg_ctx* c, T** ptr, int64_t n, const char* what) {
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  if (n <= 0) return SCCG_OK;
  hipError_t e = hipMalloc((void**)ptr, sizeof(T) * (size_t)n);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(c, SCCG_E_NOMEM, "hipMalloc(%s, %lld elements): %s", what, (long long)n, hipGetErrorString(e));
  }
  return SCCG_OK;
}

int ensure_polys(sccg_ctx* c, int which, int64_t n) {
  int64_t& cap = which ? c->capB : c->capA;
  if (n <= cap) return SCCG_OK;
  (void)hipStreamSynchronize(c->stream);
  int64_t want = n + n / 4 + 1024;
  Meta** m = which ? &c->metaB : &c->metaA;
  int64_t** ar = which ? &c->areaB : &c->areaA;
  int32_t** bg = which ? &c->bigB : &c->bigA;
  int r;
  if ((r = grow(c, m, want, "metadata")) || (r = grow(c, ar, want, "areas")) || (r = grow(c, bg, want, "big list"))) {
    cap = 0;
    return r;
  }
  cap = want;
  return SCCG_OK;
}

int ensure_pairs(sccg_ctx* c, int64_t n) {
  if (n <= c->cap_pairs) return SCCG_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  int64_t want = n + n / 4 + 1024;
  int r;
  if ((r = grow(c, &c->cls, want, "pair classes")) || (r = grow(c, &c->rec, want, "pair records")) ||
      (r = grow(c, &c->l_list, want * (kLptBuckets + 1), "pair lists")) || (r = grow(c, &c->hbox, want, "heavy boxes"))) {
    c->cap_pairs = 0;
    return r;
  }
  c->cap_pairs = want;
  return SCCG_OK;
}

// Grow a filter-stage buffer to at least n elements (waits for the stream
// before freeing the old one).
template <typename T>
int need(sccg_ctx* c, T** ptr, int64_t& cap, int64_t n, const char* what) {
  if (n <= cap && *ptr) return SCCG_OK;
  (void)hipStreamSynchronize(c->stream);
  const int64_t want = n + n / 4 + 64;
  int r = grow(c, ptr, want, what);
  cap = r ? 0 : want;
  return r;
}

int ensure_queue(sccg_ctx* c) {
  const int64_t want = (int64_t)c->p.n_queues * c->p.queue_cap;
  // The reset kernel of a call clears the slots the previous call used,
  // found from that call's head and tail counters in that call's layout, so
  // the slots are cleared here whenever the layout changes.
  if (c->queue && c->queue_slots == want && c->queue_nq == c->p.n_queues && c->queue_per == c->p.queue_cap)
    return SCCG_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (!c->queue || c->queue_slots != want) {
    int r = grow(c, &c->queue, want, "task queue");
    if (r) {
      c->queue_slots = 0;
      return r;
    }
    c->queue_slots = want;
  }
  // fresh slots must read as empty; the counters must not claim old slots
  HIP_TRY(c, hipMemsetAsync(c->queue, 0, sizeof(unsigned long long) * (size_t)want, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->st, 0, sizeof(BatchState), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->queue_nq = c->p.n_queues;
  c->queue_per = c->p.queue_cap;
  return SCCG_OK;
}

// Start/stop events for the next timed launch (created on first use).
int timing_events(sccg_ctx* c, hipEvent_t* start, hipEvent_t* stop) {
  if (c->ev_used * 2 + 2 > c->ev.size()) {
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    HIP_TRY(c, hipEventCreate(&b));
    c->ev.push_back(a);
    c->ev.push_back(b);
  }
  *start = c->ev[c->ev_used * 2];
  *stop = c->ev[c->ev_used * 2 + 1];
  c->ev_used += 1;
  return SCCG_OK;
}

int check_polys(sccg_ctx* c, const sccg_polys* P, const char* name) {
  if (!P) return fail(c, SCCG_E_ARG, "%s is NULL", name);
  if (P->n_polys < 0) return fail(c, SCCG_E_ARG, "%s.n_polys < 0", name);
  if (P->n_polys >= (int64_t)1 << 31) return fail(c, SCCG_E_ARG, "%s.n_polys >= 2^31", name);
  if (!P->offsets) return fail(c, SCCG_E_ARG, "%s.offsets is NULL", name);
  if (P->n_polys > 0 && !P->xy) return fail(c, SCCG_E_ARG, "%s.xy is NULL", name);
  return SCCG_OK;
}

Polys to_polys(const sccg_polys* P) {
  return Polys{P->n_polys, P->offsets, reinterpret_cast<const int2*>(P->xy)};
}

// ---------------------------------------------- no-allocation scratch
// Scratch of sccg_area_pairs_noalloc: one static device array per GPU,
// holding the batched state, the task queues and the per-pair arrays for at
// most kNoAllocMaxPairs pairs.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the device (kept in g_noalloc).
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 18;
constexpr int64_t kNoAllocQueueSlots = int64_t(1) << 17;  // all queues together
constexpr int kNoAllocMaxDevices = 64;
constexpr size_t na_align(size_t n) { return (n + 255) / 256 * 256; }
constexpr size_t kNaQueue = na_align(sizeof(BatchState));
constexpr size_t kNaRec = kNaQueue + na_align(sizeof(unsigned long long) * kNoAllocQueueSlots);
constexpr size_t kNaHbox = kNaRec + na_align(sizeof(PairRec) * kNoAllocMaxPairs);
constexpr size_t kNaList = kNaHbox + na_align(sizeof(Meta) * kNoAllocMaxPairs);
constexpr size_t kNaCls = kNaList + na_align(sizeof(int32_t) * (kLptBuckets + 1) * kNoAllocMaxPairs);
constexpr size_t kNoAllocBytes = kNaCls + na_align(kNoAllocMaxPairs);

struct NoAllocDevice {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this GPU
  int32_t nq = 0, cap = 0;       // queue layout of the last call (0: every slot clear)
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

__global__ void k_noalloc_clear(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Once per device, with the device current: the device address of the
// scratch array, cleared once so that every queue slot reads empty.
int noalloc_setup(sccg_ctx* c) {
  if (c->device >= kNoAllocMaxDevices) return SCCG_OK;  // the entry point reports it
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[c->device];
  if (d.ptr) return SCCG_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
  e = hipMemset(p, 0, kNoAllocBytes);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "clearing the no-allocation scratch");
  d.ptr = static_cast<unsigned char*>(p);
  d.nq = 0;
  d.cap = 0;
  return SCCG_OK;
}

}  // namespace

uint32_t* sccg::ctx_error_word(sccg_ctx* c) { return c->err; }

extern "C" {

const char* sccg_version(void) { return kVersion; }

const char* sccg_last_error(const sccg_ctx* ctx) { return ctx ? ctx->msg.c_str() : "null context"; }

int sccg_create(sccg_ctx** out, int hip_device, void* hip_stream, const sccg_params* params) {
  if (!out) return SCCG_E_ARG;
  *out = nullptr;
  sccg_ctx* c = new sccg_ctx();
  int r = resolve_params(c, params, &c->p);
  if (r) {
    delete c;
    return r;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    delete c;
    return SCCG_E_ARG;
  }
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    return SCCG_E_HIP;
  }
  (void)hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device);
  if (c->cu_count < 1) c->cu_count = 1;
  if (hipMalloc((void**)&c->err, sizeof(uint32_t)) != hipSuccess ||
      hipMalloc((void**)&c->big_count, 2 * sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void**)&c->st, sizeof(BatchState)) != hipSuccess ||
      hipMalloc((void**)&c->plain_stats, kNumStats * sizeof(unsigned long long)) != hipSuccess) {
    sccg_destroy(c);
    return SCCG_E_NOMEM;
  }
  if (hipMemset(c->err, 0, sizeof(uint32_t)) != hipSuccess || hipMemset(c->st, 0, sizeof(BatchState)) != hipSuccess ||
      hipMemset(c->plain_stats, 0, kNumStats * sizeof(unsigned long long)) != hipSuccess) {
    sccg_destroy(c);
    return SCCG_E_HIP;
  }
  if (noalloc_setup(c) != SCCG_OK) {
    sccg_destroy(c);
    return SCCG_E_HIP;
  }
  *out = c;
  return SCCG_OK;
}

int sccg_destroy(sccg_ctx* c) {
  if (!c) return SCCG_E_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  void* ptrs[] = {c->metaA,  c->areaA,  c->bigA,        c->metaB,  c->areaB,   c->bigB,    c->big_count,
                  c->err,    c->cls,    c->rec,         c->l_list, c->hbox,    c->st,      c->queue,
                  c->plain_stats, c->wave_t,
                  c->j_bbox, c->j_grid, c->j_cells,     c->j_cell_base, c->j_sums, c->j_count, c->j_start,
                  c->j_list, c->j_bcount, c->j_bstart, c->j_acc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
  return SCCG_OK;
}

int sccg_set_params(sccg_ctx* c, const sccg_params* params) {
  if (!c) return SCCG_E_ARG;
  sccg_params p;
  int r = resolve_params(c, params, &p);
  if (r) return r;
  c->p = p;
  drop_graph(c);
  return SCCG_OK;
}

int sccg_get_params(const sccg_ctx* c, sccg_params* out) {
  if (!c || !out) return SCCG_E_ARG;
  *out = c->p;
  return SCCG_OK;
}

int sccg_reserve(sccg_ctx* c, int64_t na, int64_t nb, int64_t np) {
  if (!c || na < 0 || nb < 0 || np < 0) return c ? fail(c, SCCG_E_ARG, "negative reserve size") : SCCG_E_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  int r;
  if ((r = ensure_polys(c, 0, na)) || (r = ensure_polys(c, 1, nb)) || (r = ensure_pairs(c, np)) ||
      (r = ensure_queue(c)))
    return r;
  return SCCG_OK;
}

int sccg_set_stats(sccg_ctx* c, int enable) {
  if (!c) return SCCG_E_ARG;
  if (enable & ~3) return fail(c, SCCG_E_ARG, "unknown stats flags 0x%x", enable);
  c->stats_on = enable & 1;
  c->stamps_on = (enable >> 1) & 1;
  drop_graph(c);
  return SCCG_OK;
}

int64_t sccg_get_wave_times(sccg_ctx* c, int kernel, int64_t* out, int64_t max_waves) {
  if (!c) return SCCG_E_ARG;
  if (kernel < 0 || kernel >= kStampedKernels) return fail(c, SCCG_E_ARG, "kernel %d outside [0, 2]", kernel);
  if (max_waves < 0 || (max_waves > 0 && !out)) return fail(c, SCCG_E_ARG, "NULL output or max_waves < 0");
  if (!c->wave_t || c->wave_n[kernel] == 0) return 0;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n = std::min(max_waves, c->wave_n[kernel]);
  if (n > 0)
    HIP_TRY(c, hipMemcpy(out, c->wave_t + 2 * (size_t)kernel * (size_t)c->wave_cap,
                         2 * sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost));
  return c->wave_n[kernel];
}

int sccg_set_timing(sccg_ctx* c, int enable) {
  if (!c) return SCCG_E_ARG;
  c->timing_on = enable ? 1 : 0;
  c->ev_used = 0;
  return SCCG_OK;
}

int sccg_get_timing(sccg_ctx* c, double* out_ms, int64_t* out_launches) {
  if (!c || !out_ms || !out_launches) return c ? fail(c, SCCG_E_ARG, "NULL output") : SCCG_E_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    total += ms;
  }
  *out_ms = total;
  *out_launches = (int64_t)c->ev_used;
  c->ev_used = 0;
  return SCCG_OK;
}

int sccg_get_stats(sccg_ctx* c, int64_t* out, int n) {
  if (!c || !out || n < 0) return SCCG_E_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned long long v[kNumStats] = {0};
  if (c->last_mode == SCCG_BATCHED) {
    HIP_TRY(c, hipMemcpy(v, c->st->stats, sizeof(v), hipMemcpyDeviceToHost));
  } else {
    HIP_TRY(c, hipMemcpy(v, c->plain_stats, sizeof(v), hipMemcpyDeviceToHost));
  }
  const int m = n < kNumStats ? n : kNumStats;
  for (int k = 0; k < m; ++k) out[k] = (int64_t)v[k];
  return m;
}

__global__ void k_zero_stats(unsigned long long* s) {
  if ((int)threadIdx.x < kNumStats) s[threadIdx.x] = 0;
}

// The launches of one BATCHED call on the context's stream: reset, setup,
// the union sweep, the medium sweep with the prepass of the listed pairs,
// the persistent kernel.  (A prepass on a second stream beside the sweeps
// measured no faster: the union sweep holds every wave slot.)
static int launch_batch_sequence(sccg_ctx* c, const BatchArgs& ba, int sweep_grid, int medium_grid, int grid) {
  hipError_t e;
  if ((e = launch_batch_reset(ba, c->stream)) != hipSuccess) return hip_fail(c, e, "batch reset");
  if ((e = launch_batch_setup(ba, c->stream)) != hipSuccess) return hip_fail(c, e, "batch setup");
  if ((e = launch_batch_sweeps(ba, sweep_grid, medium_grid, c->p.sweep_pair_box == 2, c->stream)) != hipSuccess)
    return hip_fail(c, e, "batch sweeps");
  if ((e = launch_batch_persistent(ba, grid, c->p.waves_per_wg, c->stream)) != hipSuccess)
    return hip_fail(c, e, "batch persistent kernel");
  return SCCG_OK;
}

static int launch_batched(sccg_ctx* c, const BatchArgs& ba, int sweep_grid, int medium_grid, int grid) {
  hipError_t e;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (c->timing_on) {
    int r = timing_events(c, &t0, &t1);
    if (r) return r;
    HIP_TRY(c, hipEventRecord(t0, c->stream));
  }
  if (int r = launch_batch_sequence(c, ba, sweep_grid, medium_grid, grid)) return r;
  if (c->timing_on) HIP_TRY(c, hipEventRecord(t1, c->stream));
  return SCCG_OK;
}

int sccg_area_pairs(sccg_ctx* c, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs, const int32_t* pair_a,
                    const int32_t* pair_b, int64_t* out_inter, int64_t* out_union, uint32_t mode) {
  if (!c) return SCCG_E_ARG;
  int r;
  if ((r = check_polys(c, A, "A")) || (r = check_polys(c, B, "B"))) return r;
  if (n_pairs < 0) return fail(c, SCCG_E_ARG, "n_pairs < 0");
  if (n_pairs >= (int64_t)1 << 31) return fail(c, SCCG_E_ARG, "n_pairs >= 2^31");
  if (mode != SCCG_PLAIN && mode != SCCG_BATCHED) return fail(c, SCCG_E_ARG, "unknown mode %u", mode);
  if (n_pairs == 0) return SCCG_OK;
  if (!pair_a || !pair_b || !out_inter || !out_union) return fail(c, SCCG_E_ARG, "NULL pair or output array");
  HIP_TRY(c, hipSetDevice(c->device));
  c->last_mode = mode;
  if (mode == SCCG_PLAIN) {
    if ((r = ensure_polys(c, 0, A->n_polys)) || (r = ensure_polys(c, 1, B->n_polys))) return r;
    hipError_t e;
    if ((e = launch_poly_meta(to_polys(A), c->metaA, c->areaA, c->bigA, c->big_count, c->err, c->stream)) !=
        hipSuccess)
      return hip_fail(c, e, "poly meta A");
    if ((e = launch_poly_meta(to_polys(B), c->metaB, c->areaB, c->bigB, c->big_count + 1, c->err, c->stream)) !=
        hipSuccess)
      return hip_fail(c, e, "poly meta B");
    PlainArgs a{};
    a.A = to_polys(A);
    a.B = to_polys(B);
    a.metaA = c->metaA;
    a.metaB = c->metaB;
    a.areaA = c->areaA;
    a.areaB = c->areaB;
    a.n_pairs = n_pairs;
    a.pa = pair_a;
    a.pb = pair_b;
    a.inter = out_inter;
    a.uni = out_union;
    a.err = c->err;
    a.stats = c->stats_on ? c->plain_stats : nullptr;
    a.box_threshold = c->p.box_threshold;
    a.gx = c->p.split_gx;
    a.gy = c->p.split_gy;
    a.lds_vertex_cap = c->p.lds_vertex_cap;
    if (c->stats_on) hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, c->stream, c->plain_stats);
    int grid = c->p.grid;
    if (grid == 0) grid = c->cu_count * plain_occupancy(c->p.wg_size, c->p.lds_vertex_cap);
    if ((int64_t)grid > n_pairs) grid = (int)n_pairs;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (c->timing_on) {
      if ((r = timing_events(c, &t0, &t1))) return r;
      HIP_TRY(c, hipEventRecord(t0, c->stream));
    }
    if ((e = launch_plain(a, c->p.wg_size, grid, c->stream)) != hipSuccess) return hip_fail(c, e, "plain kernel");
    if (c->timing_on) HIP_TRY(c, hipEventRecord(t1, c->stream));
    return SCCG_OK;
  }
  // batched
  if ((r = ensure_pairs(c, n_pairs)) || (r = ensure_queue(c))) return r;
  BatchArgs ba{};
  ba.A = to_polys(A);
  ba.B = to_polys(B);
  ba.n_pairs = n_pairs;
  ba.pa = pair_a;
  ba.pb = pair_b;
  ba.inter = out_inter;
  ba.uni = out_union;
  ba.err = c->err;
  ba.cls = c->cls;
  ba.rec = c->rec;
  ba.l_list = c->l_list;
  ba.m_list = c->l_list + (size_t)kLptBuckets * (size_t)n_pairs;
  ba.hbox = c->hbox;
  ba.st = c->st;
  ba.queue = c->queue;
  ba.queue_cap = c->p.queue_cap;
  ba.n_queues = c->p.n_queues;
  ba.chunk = c->p.queue_chunk;
  ba.heavy_verts = c->p.heavy_verts;
  ba.min_cells_to_queue = c->p.min_queue_cells;
  ba.min_classify_cells = c->p.min_classify_cells;
  ba.flags = c->p.flags;
  ba.stats_on = c->stats_on;
  int grid = c->p.grid;
  if (grid == 0) grid = c->cu_count * batch_occupancy(c->p.waves_per_wg);
  const int sweep_grid = c->cu_count * batch_sweep_occupancy(c->p.sweep_pair_box == 2);
  const int medium_grid = c->cu_count * batch_medium_occupancy();
  if (c->stamps_on) {
    // every wave of the sweeps and of the persistent kernel stamps its start and end
    const int64_t sweep_waves = (int64_t)sweep_grid * batch_sweep_waves_per_wg();
    const int64_t medium_waves = (int64_t)medium_grid * batch_sweep_waves_per_wg();
    const int64_t run_waves = (int64_t)grid * c->p.waves_per_wg;
    const int64_t want = std::max(std::max(sweep_waves, medium_waves), run_waves);
    if (want > c->wave_cap) {
      (void)hipStreamSynchronize(c->stream);
      drop_graph(c);
      if ((r = grow(c, &c->wave_t, 2 * kStampedKernels * want, "wave stamps"))) {
        c->wave_cap = 0;
        return r;
      }
      c->wave_cap = want;
    }
    ba.wave_t = c->wave_t;
    ba.wave_cap = (int32_t)c->wave_cap;
    c->wave_n[0] = sweep_waves;
    c->wave_n[1] = medium_waves;
    c->wave_n[2] = run_waves;
  }
  const bool use_graph = c->stream != nullptr && !(c->p.flags & SCCG_F_NO_GRAPH) && !c->timing_on;
  if (!use_graph) return launch_batched(c, ba, sweep_grid, medium_grid, grid);
  // the graph is keyed on every launch argument
  char key[512];
  snprintf(key, sizeof(key), "%lld/%p/%p|%lld/%p/%p|%lld/%p/%p/%p/%p|%d/%d/%d/%d/%d/%d/%u/%d/%d/%d",
           (long long)A->n_polys, (const void*)A->offsets, (const void*)A->xy,
           (long long)B->n_polys, (const void*)B->offsets, (const void*)B->xy, (long long)n_pairs,
           (const void*)pair_a, (const void*)pair_b, (void*)out_inter, (void*)out_union, ba.queue_cap, ba.n_queues,
           ba.chunk, ba.heavy_verts, ba.min_cells_to_queue, ba.min_classify_cells, ba.flags, ba.stats_on | (c->stamps_on << 1), grid,
           c->p.sweep_pair_box);
  if (!c->gexec || c->gkey != key) {
    drop_graph(c);
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    r = launch_batched(c, ba, sweep_grid, medium_grid, grid);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (r) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(c, e, "hipGraphInstantiate");
    }
    c->gkey = key;
  }
  HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
  c->graph_launches += 1;
  return SCCG_OK;
}

int sccg_area_pairs_noalloc(sccg_ctx* c, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter, int64_t* out_union) {
  if (!c) return SCCG_E_ARG;
  int r;
  if ((r = check_polys(c, A, "A")) || (r = check_polys(c, B, "B"))) return r;
  if (n_pairs < 0) return fail(c, SCCG_E_ARG, "n_pairs < 0");
  if (n_pairs > kNoAllocMaxPairs)
    return fail(c, SCCG_E_ARG, "n_pairs %lld above the no-allocation limit of %lld pairs", (long long)n_pairs,
                (long long)kNoAllocMaxPairs);
  if (n_pairs == 0) return SCCG_OK;
  if (!pair_a || !pair_b || !out_inter || !out_union) return fail(c, SCCG_E_ARG, "NULL pair or output array");
  if (c->device >= kNoAllocMaxDevices)
    return fail(c, SCCG_E_ARG, "device %d above the no-allocation limit of %d devices", c->device,
                kNoAllocMaxDevices);
  HIP_TRY(c, hipSetDevice(c->device));
  const int32_t nq = c->p.n_queues;
  const int32_t cap = (int32_t)std::min<int64_t>(c->p.queue_cap, kNoAllocQueueSlots / nq);
  unsigned char* base;
  {
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    NoAllocDevice& d = g_noalloc[c->device];
    if (!d.ptr) return fail(c, SCCG_E_HIP, "no-allocation scratch not set up on device %d", c->device);
    base = d.ptr;
    // the reset kernel clears the slots the previous call used in that
    // call's layout: a new layout needs every slot cleared first
    if (d.nq != 0 && (d.nq != nq || d.cap != cap)) {
      hipLaunchKernelGGL(k_noalloc_clear, dim3(256), dim3(256), 0, c->stream,
                         reinterpret_cast<unsigned long long*>(base + kNaQueue), (int64_t)kNoAllocQueueSlots);
      HIP_TRY(c, hipGetLastError());
    }
    d.nq = nq;
    d.cap = cap;
  }
  BatchArgs ba{};
  ba.A = to_polys(A);
  ba.B = to_polys(B);
  ba.n_pairs = n_pairs;
  ba.pa = pair_a;
  ba.pb = pair_b;
  ba.inter = out_inter;
  ba.uni = out_union;
  ba.err = c->err;
  ba.st = reinterpret_cast<BatchState*>(base);
  ba.queue = reinterpret_cast<unsigned long long*>(base + kNaQueue);
  ba.rec = reinterpret_cast<PairRec*>(base + kNaRec);
  ba.hbox = reinterpret_cast<Meta*>(base + kNaHbox);
  ba.l_list = reinterpret_cast<int32_t*>(base + kNaList);
  ba.m_list = ba.l_list + (size_t)kLptBuckets * (size_t)n_pairs;
  ba.cls = base + kNaCls;
  ba.queue_cap = cap;
  ba.n_queues = nq;
  ba.chunk = c->p.queue_chunk;
  ba.heavy_verts = c->p.heavy_verts;
  ba.min_cells_to_queue = c->p.min_queue_cells;
  ba.min_classify_cells = c->p.min_classify_cells;
  ba.flags = c->p.flags;
  ba.stats_on = 0;
  int grid = c->p.grid;
  if (grid == 0) grid = c->cu_count * batch_occupancy(c->p.waves_per_wg);
  const int sweep_grid = c->cu_count * batch_sweep_occupancy(c->p.sweep_pair_box == 2);
  const int medium_grid = c->cu_count * batch_medium_occupancy();
  return launch_batch_sequence(c, ba, sweep_grid, medium_grid, grid);
}

int sccg_jaccard_sets(sccg_ctx* c, int64_t n_sets, const int64_t* set_pair_off, const int64_t* inter,
                      const int64_t* uni, uint32_t flags, int64_t* out_sum_i, int64_t* out_sum_u,
                      int64_t* out_n_contrib, double* out_j, double* out_jprime) {
  if (!c) return SCCG_E_ARG;
  if (n_sets < 0) return fail(c, SCCG_E_ARG, "n_sets < 0");
  if (flags & ~SCCG_J_INCLUDE_ZERO) return fail(c, SCCG_E_ARG, "unknown Jaccard flags 0x%x", flags);
  if (n_sets == 0) return SCCG_OK;
  if (!set_pair_off || !inter || !uni || !out_sum_i || !out_sum_u || !out_n_contrib || !out_j)
    return fail(c, SCCG_E_ARG, "NULL array");
  HIP_TRY(c, hipSetDevice(c->device));
  int r;
  // one accumulator per set, and past them the chunk counter
  if ((r = need(c, &c->j_acc, c->j_cap[8], n_sets + 1, "set accumulators"))) return r;
  const int grid = c->cu_count * 4;
  hipError_t e = launch_jaccard(n_sets, set_pair_off, inter, uni, flags, out_sum_i, out_sum_u, out_n_contrib, out_j,
                                out_jprime, c->j_acc, &c->j_acc[n_sets].si, grid, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "jaccard");
  return SCCG_OK;
}

int sccg_join_sets(sccg_ctx* c, const sccg_polys* A, const sccg_polys* B, int64_t n_sets, const int64_t* a_set_off,
                   const int64_t* b_set_off, int32_t cell, int64_t cap, int32_t* out_pa, int32_t* out_pb,
                   int64_t* out_set_off, int64_t* out_total) {
  if (!c) return SCCG_E_ARG;
  int r;
  if ((r = check_polys(c, A, "A")) || (r = check_polys(c, B, "B"))) return r;
  if (n_sets < 0) return fail(c, SCCG_E_ARG, "n_sets < 0");
  if (cap < 0) return fail(c, SCCG_E_ARG, "cap < 0");
  if (cell == 0) cell = 64;
  if (cell < 1 || cell > (1 << 20)) return fail(c, SCCG_E_ARG, "cell outside [1, 2^20]");
  if (!out_total || !out_set_off || (n_sets > 0 && (!a_set_off || !b_set_off)))
    return fail(c, SCCG_E_ARG, "NULL offsets or output");
  if (cap > 0 && (!out_pa || !out_pb)) return fail(c, SCCG_E_ARG, "NULL pair output with cap > 0");
  HIP_TRY(c, hipSetDevice(c->device));
  *out_total = 0;
  if (n_sets == 0) {
    HIP_TRY(c, hipMemsetAsync(out_set_off, 0, sizeof(int64_t), c->stream));
    return SCCG_OK;
  }
  hipError_t e;
  const Polys pA = to_polys(A), pB = to_polys(B);
  if ((r = ensure_polys(c, 0, A->n_polys)) || (r = ensure_polys(c, 1, B->n_polys))) return r;
  if ((e = launch_poly_meta(pA, c->metaA, c->areaA, c->bigA, c->big_count, c->err, c->stream)) != hipSuccess)
    return hip_fail(c, e, "poly meta A");
  if ((e = launch_poly_meta(pB, c->metaB, c->areaB, c->bigB, c->big_count + 1, c->err, c->stream)) != hipSuccess)
    return hip_fail(c, e, "poly meta B");
  // grids: per-set extents of A, cells per set, their offsets
  if ((r = need(c, &c->j_bbox, c->j_cap[0], n_sets, "join boxes")) ||
      (r = need(c, &c->j_grid, c->j_cap[1], n_sets, "join grids")) ||
      (r = need(c, &c->j_cells, c->j_cap[2], n_sets, "join cells")) ||
      (r = need(c, &c->j_cell_base, c->j_cap[3], n_sets + 1, "join cell offsets")) ||
      (r = need(c, &c->j_sums, c->j_cap[4], scan_scratch(n_sets), "scan sums")))
    return r;
  if ((e = launch_join_grid(pA, c->metaA, a_set_off, n_sets, cell, c->j_bbox, c->j_grid, c->j_cells, c->j_cell_base,
                            c->j_sums, c->err, c->stream)) != hipSuccess)
    return hip_fail(c, e, "join grid");
  int64_t n_cells = 0;
  HIP_TRY(c, hipMemcpyAsync(&n_cells, c->j_cell_base + n_sets, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // counting sort of (cell, A polygon) entries
  if ((r = need(c, &c->j_count, c->j_cap[5], n_cells + 1, "cell counts")) ||
      (r = need(c, &c->j_start, c->j_cap[6], n_cells + 1, "cell starts")) ||
      (r = need(c, &c->j_sums, c->j_cap[4], scan_scratch(n_cells), "scan sums")))
    return r;
  HIP_TRY(c, hipMemsetAsync(c->j_count, 0, sizeof(int32_t) * (size_t)(n_cells + 1), c->stream));
  if ((e = launch_join_cells(pA, c->metaA, a_set_off, n_sets, c->j_grid, c->j_cell_base, cell, 0, c->j_count,
                             nullptr, nullptr, c->stream)) != hipSuccess ||
      (e = launch_join_scan_counts(c->j_count, n_cells, c->j_start, c->j_sums, c->stream)) != hipSuccess)
    return hip_fail(c, e, "join cell counts");
  int64_t n_entries = 0;
  HIP_TRY(c, hipMemcpyAsync(&n_entries, c->j_start + n_cells, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if ((r = need(c, &c->j_list, c->j_cap[7], n_entries + 1, "cell lists"))) return r;
  HIP_TRY(c, hipMemsetAsync(c->j_count, 0, sizeof(int32_t) * (size_t)(n_cells + 1), c->stream));
  if ((e = launch_join_cells(pA, c->metaA, a_set_off, n_sets, c->j_grid, c->j_cell_base, cell, 1, c->j_count,
                             c->j_start, c->j_list, c->stream)) != hipSuccess)
    return hip_fail(c, e, "join cell lists");
  // pairs: count per B polygon, offsets, then (if they fit) write and sort
  if ((r = need(c, &c->j_bcount, c->j_cap[8], B->n_polys + 1, "pair counts")) ||
      (r = need(c, &c->j_bstart, c->j_cap[9], B->n_polys + 1, "pair starts")) ||
      (r = need(c, &c->j_sums, c->j_cap[4], scan_scratch(B->n_polys), "scan sums")))
    return r;
  if ((e = launch_join_pairs(pB, c->metaA, c->metaB, b_set_off, n_sets, c->j_grid, c->j_cell_base, c->j_start,
                             c->j_list, cell, 0, c->j_bcount, nullptr, 0, nullptr, nullptr, c->stream)) != hipSuccess ||
      (e = launch_join_scan_counts(c->j_bcount, B->n_polys, c->j_bstart, c->j_sums, c->stream)) != hipSuccess)
    return hip_fail(c, e, "join pair counts");
  int64_t total = 0;
  HIP_TRY(c, hipMemcpyAsync(&total, c->j_bstart + B->n_polys, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *out_total = total;
  if (total <= cap && total > 0) {
    if ((e = launch_join_pairs(pB, c->metaA, c->metaB, b_set_off, n_sets, c->j_grid, c->j_cell_base, c->j_start,
                               c->j_list, cell, 1, nullptr, c->j_bstart, cap, out_pa, out_pb, c->stream)) != hipSuccess)
      return hip_fail(c, e, "join pairs");
  }
  if ((e = launch_join_set_off(n_sets, B->n_polys, b_set_off, c->j_bstart, out_set_off, c->stream)) != hipSuccess)
    return hip_fail(c, e, "join set offsets");
  return SCCG_OK;
}

int sccg_relate_pairs(sccg_ctx* c, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs, const int32_t* pair_a,
                      const int32_t* pair_b, const int64_t* inter, uint32_t* out_rel) {
  if (!c) return SCCG_E_ARG;
  int r;
  if ((r = check_polys(c, A, "A")) || (r = check_polys(c, B, "B"))) return r;
  if (n_pairs < 0) return fail(c, SCCG_E_ARG, "n_pairs < 0");
  if (n_pairs == 0) return SCCG_OK;
  if (!pair_a || !pair_b || !inter || !out_rel) return fail(c, SCCG_E_ARG, "NULL pair, count or output array");
  HIP_TRY(c, hipSetDevice(c->device));
  if ((r = ensure_polys(c, 0, A->n_polys)) || (r = ensure_polys(c, 1, B->n_polys))) return r;
  hipError_t e;
  const Polys pA = to_polys(A), pB = to_polys(B);
  if ((e = launch_poly_meta(pA, c->metaA, c->areaA, c->bigA, c->big_count, c->err, c->stream)) != hipSuccess ||
      (e = launch_poly_meta(pB, c->metaB, c->areaB, c->bigB, c->big_count + 1, c->err, c->stream)) != hipSuccess)
    return hip_fail(c, e, "poly meta");
  if ((e = launch_relate(pA, pB, c->metaA, c->metaB, c->areaA, c->areaB, n_pairs, pair_a, pair_b, inter, out_rel,
                         c->err, c->stream)) != hipSuccess)
    return hip_fail(c, e, "relate");
  return SCCG_OK;
}

int sccg_validate_polys(sccg_ctx* c, const sccg_polys* P, int64_t* out_first_bad) {
  if (!c) return SCCG_E_ARG;
  int r = check_polys(c, P, "P");
  if (r) return r;
  if (!out_first_bad) return fail(c, SCCG_E_ARG, "out_first_bad is NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  hipError_t e = launch_validate(to_polys(P), out_first_bad, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "validate");
  return SCCG_OK;
}

int64_t sccg_graph_launches(const sccg_ctx* c) { return c ? c->graph_launches : -1; }

int sccg_valu_peak(sccg_ctx* c, int32_t iters, double* out_lane_ops_per_s, double* out_ms) {
  if (!c) return SCCG_E_ARG;
  if (iters < 1 || iters > (1 << 24)) return fail(c, SCCG_E_ARG, "iters outside [1, 2^24]");
  if (!out_lane_ops_per_s || !out_ms) return fail(c, SCCG_E_ARG, "NULL output");
  HIP_TRY(c, hipSetDevice(c->device));
  int r;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((r = timing_events(c, &t0, &t1))) return r;
  c->ev_used -= 1;  // the pair is borrowed, not counted as a timed launch
  const int grid = c->cu_count * 8;  // 8 waves per SIMD
  hipError_t e;
  // one untimed launch brings the clocks up, then the timed one
  if ((e = launch_valu_peak(grid, iters, c->plain_stats, c->stream)) != hipSuccess) return hip_fail(c, e, "valu peak");
  HIP_TRY(c, hipEventRecord(t0, c->stream));
  if ((e = launch_valu_peak(grid, iters, c->plain_stats, c->stream)) != hipSuccess) return hip_fail(c, e, "valu peak");
  HIP_TRY(c, hipEventRecord(t1, c->stream));
  HIP_TRY(c, hipEventSynchronize(t1));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, t0, t1));
  *out_ms = ms;
  *out_lane_ops_per_s = (double)grid * 256.0 * (double)iters * 32.0 / ((double)ms * 1e-3);
  return SCCG_OK;
}

int sccg_sync(sccg_ctx* c) {
  if (!c) return SCCG_E_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint32_t err = 0;
  HIP_TRY(c, hipMemcpy(&err, c->err, sizeof(err), hipMemcpyDeviceToHost));
  if (err) HIP_TRY(c, hipMemset(c->err, 0, sizeof(err)));
  if (err & kErrWatchdog) return fail(c, SCCG_E_DEVICE, "device watchdog: a bounded wait ran out (error word 0x%x)", err);
  if (err & (kErrIndex | kErrSide | kErrCoord))
    return fail(c, SCCG_E_RANGE, "device range error:%s%s%s", (err & kErrIndex) ? " pair index out of range" : "",
                (err & kErrSide) ? " pair-box side above 32767" : "",
                (err & kErrCoord) ? " coordinate magnitude above 2^30" : "");
  return SCCG_OK;
}

}  // extern "C"
