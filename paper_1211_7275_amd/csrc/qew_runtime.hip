// qew_runtime.hip -- host runtime and C ABI of libqew (declared in include/qew.h).
//
// A plan holds the validated problem, the per-sample offsets of the state
// buffers, two tile work lists (measurement / one-step tiles of fixed size,
// and fused workgroup tiles whose valid width depends on the blocking depth k),
// and the layout of the caller's workspace.  qew_run walks the measurement
// steps: at each one it reduces Eqs. (3)-(5) of the state (and, when the
// problem asks for it, the structure factor of Eq. (6)), and between them
// it advances the chains by Euler steps (Eq. (1), Sec. III B), one or k steps
// per launch, replaying captured hipGraphs of 16 launches where it can.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qew.h"
#include "qew_internal.hpp"

using namespace qew;

// Scratch of qew_run_noalloc: the plan's tables, tile lists, measurement
// partials and series, for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel or copy: it uses the device
// address that hipGetSymbolAddress returns, fetched once per device.  Calls
// of qew_run_noalloc on one GPU share the array, so calls that overlap on
// one GPU race (each call rewrites tables, flags and series before use).
static constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

qew_status fail(qew_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define QEW_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(QEW_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

constexpr int64_t kMaxL = int64_t(1) << 30;
constexpr int kGraphLaunches = 16;
constexpr int64_t kSqChunk = 4096;  // modes per binning chunk
constexpr int kTuneTiles[5] = {1024, 1536, 2048, 3072, 4096};
constexpr int kTuneK[6] = {16, 32, 48, 56, 64, 96};
// The fused path runs stretches shorter than this with the one-step kernel:
// a fused launch moves the state and its node cache through HBM (48 B per
// site) however few steps it takes, while a one-step launch moves 16 B per
// site and its first step also takes the measurement the stretch starts
// with.  The node cache is rebuilt before the next fused launch.
constexpr int64_t kShortStretch = 4;
// The fused path switches to its sparse variant when the cell changes expected
// per wave and sub-step (a wave holds 64 P sites) fall below this: most
// sub-steps of a wave then have no cell change at all.
constexpr double kSparseRequestsPerWave = 0.5;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t err, off, L, f, f32, did, mt_s, mt_p0, mt_len, mt_first, ft_s, ft_p0, ft_len, sq_chunk_lo,
      sq_chunk_first;
  size_t tables_end;
  size_t part, series, ens;
  size_t small_end;  // end of the tables, partials and series (the regions qew_run_noalloc keeps in scratch)
  size_t sq_series, sq_part, fftA, fftB, stA0, stA1, stB0, stB1, ndA, ndB;
  size_t total;
};

// A captured sequence of kGraphLaunches stepping launches.  A plan keeps one
// per kernel variant (fused: dense and sparse; one-step: slot 0), so a
// variant switch inside a run never destroys a graph that may still be
// queued.  An entry is replaced only when its workspace or geometry changed,
// which happens between runs, after qew_run has drained its stream.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  int key_k = -1, key_tile = -1, key_grid = -1;
};

}  // namespace

struct qew_plan_s {
  // problem
  int32_t S = 0, kind = 0, precision = 0, path = 0, k_req = 0, tile_req = 0, flags = 0, period = 0;
  int32_t sq_bins = 0;
  std::vector<int64_t> sq_edges;
  std::vector<int32_t> sq_chunk_lo;     // [n_chunks + 1] mode ranges of the binning chunks
  std::vector<int32_t> sq_chunk_first;  // [sq_bins + 1] first chunk of each bin
  double c = 0, dt = 0, strength = 0;
  uint64_t seed = 0;
  int64_t n_steps = 0;
  std::vector<int64_t> L, meas;
  std::vector<double> f;
  std::vector<uint32_t> did;
  // derived
  std::vector<int64_t> off;
  int64_t padded = 0, total_sites = 0;
  std::vector<int32_t> mt_s, mt_p0, mt_len, mt_first;
  std::vector<int32_t> ft_s, ft_p0, ft_len;
  int32_t ft_capacity = 0;
  int32_t k = 1, tile = 0, autotuned = 0;
  Layout lay{};
  std::vector<char> table_img;  // host image of the table region (current tile lists)
  // run state
  char* small_base = nullptr;  // during qew_run_noalloc: base of the small regions (the scratch array)
  bool direct_only = false;    // during qew_run_noalloc: no graphs, events or host readbacks
  int64_t cur_step = 0;
  int cur_buf = 0;
  void* state_ws = nullptr;
  bool nodes_valid = false;
  int fused_grid = 0;
  hipStream_t cap_stream = nullptr;
  GraphCache graph[2];
  qew_run_stats stats{};
  // fused variant: sparse (1) or dense (0), chosen from the velocities of the
  // measurement before last (two readback slots used in turn)
  int sparse = 0;
  int rb_next = 0;                              // slot of the next readback
  bool rb_valid[2] = {false, false};            // the slot holds a readback not yet used
  double* rb_host = nullptr;                    // [2][S] pinned: v of every sample
  hipEvent_t rb_event[2] = {nullptr, nullptr};  // complete when the slot holds its velocities
};

namespace {

bool fused(const qew_plan_t* p) { return p->path == QEW_FUSED; }

void refresh_table_image(qew_plan_t* p);

void build_fused_tiles(qew_plan_t* p, int tile, int k) {
  p->ft_s.clear();
  p->ft_p0.clear();
  p->ft_len.clear();
  const int64_t V = tile - 2 * k;
  for (int32_t s = 0; s < p->S; ++s) {
    const int64_t L = p->L[s];
    for (int64_t p0 = 0; p0 < L; p0 += V) {
      p->ft_s.push_back(s);
      p->ft_p0.push_back((int32_t)p0);
      p->ft_len.push_back((int32_t)std::min<int64_t>(V, L - p0));
    }
  }
  p->k = k;
  p->tile = tile;
  if (p->lay.total) refresh_table_image(p);
}

int64_t fused_tile_count(const qew_plan_t* p, int tile, int k) {
  const int64_t V = tile - 2 * k;
  int64_t n = 0;
  for (int64_t L : p->L) n += (L + V - 1) / V;
  return n;
}

void compute_layout(qew_plan_t* p) {
  Layout& l = p->lay;
  const size_t S = (size_t)p->S;
  const size_t nmt = p->mt_s.size();
  const size_t nft = (size_t)p->ft_capacity;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  l.err = take(4);
  l.off = take(S * 8);
  l.L = take(S * 4);
  l.f = take(S * 8);
  l.f32 = take(S * 4);
  l.did = take(S * 4);
  l.mt_s = take(nmt * 4);
  l.mt_p0 = take(nmt * 4);
  l.mt_len = take(nmt * 4);
  l.mt_first = take((S + 1) * 4);
  l.ft_s = take(nft * 4);
  l.ft_p0 = take(nft * 4);
  l.ft_len = take(nft * 4);
  l.sq_chunk_lo = take(p->sq_chunk_lo.size() * 4);
  l.sq_chunk_first = take(p->sq_chunk_first.size() * 4);
  l.tables_end = o;
  l.part = take(nmt * sizeof(Partial));
  l.series = take(S * std::max<size_t>(p->meas.size(), 1) * 3 * 8);
  l.ens = take(7 * std::max<size_t>(p->meas.size(), 1) * 8);
  l.small_end = o;
  if (p->sq_bins > 0) {
    const size_t half = (size_t)(p->L[0] / 2);
    l.sq_series = take(std::max<size_t>(p->meas.size(), 1) * p->sq_bins * 8);
    l.sq_part = take(p->sq_chunk_lo.size() * 8);
    l.fftA = take(S * half * 16 + (half + 1) * 8);  // either buffer may hold S_n and the mean
    l.fftB = take(S * half * 16 + (half + 1) * 8);  // also holds the per-mode mean
  } else {
    l.sq_series = l.sq_part = l.fftA = l.fftB = 0;
  }
  const size_t n = (size_t)p->padded;
  if (p->precision == QEW_FP64_PLAIN) {
    l.stA0 = take(n * 8);
    l.stA1 = 0;
    l.stB0 = take(n * 8);
    l.stB1 = 0;
  } else {
    l.stA0 = take(n * 4);
    l.stA1 = take(n * 4);
    l.stB0 = take(n * 4);
    l.stB1 = take(n * 4);
  }
  if (fused(p)) {
    l.ndA = take(n * 16);
    l.ndB = take(n * 16);
  } else {
    l.ndA = l.ndB = 0;
  }
  l.total = o;
}

// Base of the small regions (tables, partials, series): the workspace, or the
// scratch array during qew_run_noalloc.  The state buffers are always in the
// workspace.
char* small_of(const qew_plan_t* p, void* ws) {
  return p->small_base ? p->small_base : static_cast<char*>(ws);
}

Tables tables_of(const qew_plan_t* p, void* ws) {
  char* b = small_of(p, ws);
  const Layout& l = p->lay;
  Tables t;
  t.off = reinterpret_cast<const int64_t*>(b + l.off);
  t.L = reinterpret_cast<const int32_t*>(b + l.L);
  t.f = reinterpret_cast<const double*>(b + l.f);
  t.f32 = reinterpret_cast<const float*>(b + l.f32);
  t.did = reinterpret_cast<const uint32_t*>(b + l.did);
  t.mt_s = reinterpret_cast<const int32_t*>(b + l.mt_s);
  t.mt_p0 = reinterpret_cast<const int32_t*>(b + l.mt_p0);
  t.mt_len = reinterpret_cast<const int32_t*>(b + l.mt_len);
  t.mt_first = reinterpret_cast<const int32_t*>(b + l.mt_first);
  t.ft_s = reinterpret_cast<const int32_t*>(b + l.ft_s);
  t.ft_p0 = reinterpret_cast<const int32_t*>(b + l.ft_p0);
  t.ft_len = reinterpret_cast<const int32_t*>(b + l.ft_len);
  t.n_mt = (int32_t)p->mt_s.size();
  t.n_ft = (int32_t)p->ft_s.size();
  t.err = reinterpret_cast<int*>(b + l.err);
  return t;
}

Phys phys_of(const qew_plan_t* p) {
  Phys ph;
  ph.c = p->c;
  ph.dt = p->dt;
  ph.strength = p->strength;
  ph.cf = (float)p->c;
  ph.dtf = (float)p->dt;
  const bool force_values = p->kind == QEW_RF_CR_UNIFORM || p->kind == QEW_RF_PC_GAUSS;
  ph.sgn_strf = force_values ? (float)p->strength : -(float)p->strength;
  ph.k0 = (uint32_t)(p->seed & 0xffffffffu);
  ph.k1 = (uint32_t)(p->seed >> 32);
  ph.period = p->period;
  return ph;
}

double* plain_buf(const qew_plan_t* p, void* ws, int which) {
  return reinterpret_cast<double*>(static_cast<char*>(ws) + (which ? p->lay.stB0 : p->lay.stA0));
}

SplitBuf split_buf(const qew_plan_t* p, void* ws, int which) {
  char* b = static_cast<char*>(ws);
  const Layout& l = p->lay;
  SplitBuf s;
  s.cell = reinterpret_cast<int32_t*>(b + (which ? l.stB0 : l.stA0));
  s.frac = reinterpret_cast<float*>(b + (which ? l.stB1 : l.stA1));
  s.nodes = fused(p) ? reinterpret_cast<float4*>(b + (which ? l.ndB : l.ndA)) : nullptr;
  return s;
}

// Host image of the table region (offsets as laid out in the workspace), kept
// in the plan and rebuilt whenever the fused tile list changes.
void refresh_table_image(qew_plan_t* p) {
  const Layout& l = p->lay;
  std::vector<char>& img = p->table_img;
  img.assign(l.tables_end, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(img.data() + at, src, bytes);
  };
  std::vector<int32_t> L32(p->S);
  std::vector<float> f32(p->S);
  for (int s = 0; s < p->S; ++s) {
    L32[s] = (int32_t)p->L[s];
    f32[s] = (float)p->f[s];
  }
  put(l.off, p->off.data(), p->S * 8);
  put(l.L, L32.data(), p->S * 4);
  put(l.f, p->f.data(), p->S * 8);
  put(l.f32, f32.data(), p->S * 4);
  put(l.did, p->did.data(), p->S * 4);
  put(l.mt_s, p->mt_s.data(), p->mt_s.size() * 4);
  put(l.mt_p0, p->mt_p0.data(), p->mt_p0.size() * 4);
  put(l.mt_len, p->mt_len.data(), p->mt_len.size() * 4);
  put(l.mt_first, p->mt_first.data(), p->mt_first.size() * 4);
  put(l.ft_s, p->ft_s.data(), p->ft_s.size() * 4);
  put(l.ft_p0, p->ft_p0.data(), p->ft_p0.size() * 4);
  put(l.ft_len, p->ft_len.data(), p->ft_len.size() * 4);
  put(l.sq_chunk_lo, p->sq_chunk_lo.data(), p->sq_chunk_lo.size() * 4);
  put(l.sq_chunk_first, p->sq_chunk_first.data(), p->sq_chunk_first.size() * 4);
}

// Copy the plan's table image to the small regions' base (no allocation).
qew_status upload_tables(qew_plan_t* p, void* ws, hipStream_t st) {
  QEW_HIP(hipMemcpyAsync(small_of(p, ws), p->table_img.data(), p->table_img.size(), hipMemcpyHostToDevice, st));
  QEW_HIP(hipStreamSynchronize(st));
  return QEW_OK;
}

double* series_of(const qew_plan_t* p, void* ws) {
  return reinterpret_cast<double*>(small_of(p, ws) + p->lay.series);
}

// Measurements not yet taken read as NaN.
qew_status clear_series(const qew_plan_t* p, void* ws, hipStream_t st) {
  QEW_HIP(launch_fill_f64(series_of(p, ws), (int64_t)p->S * (int64_t)p->meas.size() * 3,
                          __builtin_nan(""), st));
  if (p->sq_bins > 0)
    QEW_HIP(launch_fill_f64(reinterpret_cast<double*>(static_cast<char*>(ws) + p->lay.sq_series),
                            (int64_t)p->meas.size() * p->sq_bins, __builtin_nan(""), st));
  return QEW_OK;
}

qew_status init_state(qew_plan_t* p, void* ws, hipStream_t st) {
  const Tables t = tables_of(p, ws);
  qew_status rc = clear_series(p, ws, st);
  if (rc != QEW_OK) return rc;
  if (p->precision == QEW_FP64_PLAIN) {
    QEW_HIP(launch_init_plain(t, plain_buf(p, ws, 0), st));
  } else {
    QEW_HIP(launch_init_split(t, split_buf(p, ws, 0), phys_of(p), p->kind, fused(p), st));
  }
  p->cur_buf = 0;
  p->cur_step = 0;
  p->state_ws = ws;
  p->nodes_valid = true;
  return QEW_OK;
}

Partial* partials_of(const qew_plan_t* p, void* ws) {
  return reinterpret_cast<Partial*>(small_of(p, ws) + p->lay.part);
}

// One Euler step from buffer `from` with the one-step kernel of the plan's
// precision (the split one-step kernel on the fused path); with `part`
// non-null it also writes the measurement partials of the state it reads.
hipError_t onestep_launch(const qew_plan_t* p, void* ws, int from, Partial* part, hipStream_t st) {
  const Tables t = tables_of(p, ws);
  const Phys ph = phys_of(p);
  if (p->precision == QEW_FP64_PLAIN)
    return launch_step_plain(t, plain_buf(p, ws, from), plain_buf(p, ws, from ^ 1), ph, p->kind, part, st);
  SplitBuf in = split_buf(p, ws, from), out = split_buf(p, ws, from ^ 1);
  in.nodes = out.nodes = nullptr;  // the one-step kernel regenerates nodes
  return launch_step_split1(t, in, out, ph, p->kind, part, st);
}

// One launch of the fused kernel: nsub Euler steps from buffer `from`.
hipError_t fused_launch(const qew_plan_t* p, void* ws, int from, int nsub, hipStream_t st) {
  return launch_step_fused(tables_of(p, ws), split_buf(p, ws, from), split_buf(p, ws, from ^ 1), phys_of(p),
                           p->kind, p->tile, p->k, nsub, p->fused_grid, p->sparse != 0, st);
}

// The plan's stepping launch: fused (nsub steps) on the fused path, else one step.
hipError_t step_launch(const qew_plan_t* p, void* ws, int from, int nsub, hipStream_t st) {
  if (fused(p)) return fused_launch(p, ws, from, nsub, st);
  return onestep_launch(p, ws, from, nullptr, st);
}

qew_status ensure_fused_grid(qew_plan_t* p) {
  if (!fused(p)) return QEW_OK;
  if (!fused_fits(p->tile)) return fail(QEW_EUNSUPPORTED, "tile %d needs more LDS than this device allows", p->tile);
  const int maxg = fused_max_grid(p->tile);
  if (maxg <= 0) return fail(QEW_EDEVICE, "could not query occupancy of the fused kernel");
  const int need = (int)p->ft_s.size();
  p->fused_grid = std::max(1, std::min(need, maxg));
  return QEW_OK;
}

void drop_graph(GraphCache& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g = GraphCache{};
}

// Only between runs (the stream of the last run has drained; qew_run
// synchronizes its stream before it returns, on success and on failure).
void drop_graphs(qew_plan_t* p) {
  for (GraphCache& g : p->graph) drop_graph(g);
}

// Graph of kGraphLaunches full launches of the current variant starting
// (and ending) at buffer 0.
qew_status ensure_graph(qew_plan_t* p, void* ws) {
  GraphCache& g = p->graph[fused(p) && p->sparse ? 1 : 0];
  if (g.exec && g.ws == ws && g.key_k == p->k && g.key_tile == p->tile && g.key_grid == p->fused_grid)
    return QEW_OK;
  drop_graph(g);
  if (!p->cap_stream) QEW_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  QEW_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < kGraphLaunches && le == hipSuccess; ++i)
    le = step_launch(p, ws, i & 1, p->k, p->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(p->cap_stream, &graph);
  if (le != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(QEW_EDEVICE, "graph capture failed: %s",
                hipGetErrorString(le != hipSuccess ? le : ee));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(QEW_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
  g.exec = exec;
  g.ws = ws;
  g.key_k = p->k;
  g.key_tile = p->tile;
  g.key_grid = p->fused_grid;
  return QEW_OK;
}

void count_launches(qew_plan_t* p, int64_t n, bool fused_kernel) {
  p->stats.step_launches += n;
  if (fused_kernel) {
    p->stats.fused_launches += n;
    if (p->sparse) p->stats.sparse_launches += n;
  }
}

// Advance the state by n Euler steps with the plan's stepping kernel
// (buffer parity tracked in the plan).
qew_status advance(qew_plan_t* p, void* ws, int64_t n, hipStream_t st) {
  const int kk = p->k;
  int64_t blocks = n / kk;
  const int rem = (int)(n % kk);
  const bool use_graph = !(p->flags & QEW_FLAG_NO_GRAPH) && !p->direct_only;
  const bool fk = fused(p);
  if (use_graph && blocks >= kGraphLaunches + (p->cur_buf ? 1 : 0)) {
    if (p->cur_buf) {
      QEW_HIP(step_launch(p, ws, p->cur_buf, kk, st));
      p->cur_buf ^= 1;
      count_launches(p, 1, fk);
      --blocks;
    }
    qew_status rc = ensure_graph(p, ws);
    if (rc != QEW_OK) return rc;
    const hipGraphExec_t exec = p->graph[fk && p->sparse ? 1 : 0].exec;
    while (blocks >= kGraphLaunches) {
      QEW_HIP(hipGraphLaunch(exec, st));
      blocks -= kGraphLaunches;
      count_launches(p, kGraphLaunches, fk);
      p->stats.graph_launches++;
    }
  }
  for (; blocks > 0; --blocks) {
    QEW_HIP(step_launch(p, ws, p->cur_buf, kk, st));
    p->cur_buf ^= 1;
    count_launches(p, 1, fk);
  }
  if (rem) {
    QEW_HIP(step_launch(p, ws, p->cur_buf, rem, st));
    p->cur_buf ^= 1;
    count_launches(p, 1, fk);
  }
  if (fk) p->stats.fused_steps += n;
  return QEW_OK;
}

// n Euler steps with the one-step kernel on the fused path (short stretches);
// the first one also writes the measurement partials when `part` is given.
// The node cache no longer matches the state afterwards.
qew_status advance_onestep(qew_plan_t* p, void* ws, int64_t n, Partial* part, hipStream_t st) {
  for (int64_t i = 0; i < n; ++i) {
    QEW_HIP(onestep_launch(p, ws, p->cur_buf, i == 0 ? part : nullptr, st));
    p->cur_buf ^= 1;
    count_launches(p, 1, false);
  }
  if (fused(p) && n > 0) p->nodes_valid = false;
  return QEW_OK;
}

// Fused variant for the next stretch of steps (the steps between two
// measurements), from the velocities of the measurement before last: a line
// advancing at v changes cell about v dt times per site and step.  The host
// waits for those velocities, which the device produced while the last
// stretch was still queued behind them, so the wait leaves no gap on the
// device.  A flag can force either variant.
qew_status choose_variant(qew_plan_t* p) {
  if (p->flags & QEW_FLAG_FUSED_DENSE) { p->sparse = 0; return QEW_OK; }
  if (p->flags & QEW_FLAG_FUSED_SPARSE) { p->sparse = 1; return QEW_OK; }
  const int slot = p->rb_next;
  if (!p->rb_valid[slot]) return QEW_OK;
  QEW_HIP(hipEventSynchronize(p->rb_event[slot]));
  p->rb_valid[slot] = false;
  const double* v = p->rb_host + (size_t)slot * p->S;
  double moves = 0.0;  // expected cell changes per step over all sites
  for (int s = 0; s < p->S; ++s) moves += (double)p->L[s] * std::fabs(v[s]) * p->dt;
  const double per_wave = moves / (double)std::max<int64_t>(p->total_sites, 1) * (p->tile / 4);
  p->sparse = (std::isfinite(per_wave) && per_wave < kSparseRequestsPerWave) ? 1 : 0;
  return QEW_OK;
}

// After measurement mi: send the velocities of every sample to the host
// (next slot).
qew_status post_velocities(qew_plan_t* p, void* ws, int mi, hipStream_t st) {
  const int slot = p->rb_next;
  const size_t n_meas = p->meas.size();
  const double* v = series_of(p, ws) + (size_t)mi * 3;
  QEW_HIP(hipMemcpy2DAsync(p->rb_host + (size_t)slot * p->S, sizeof(double), v, n_meas * 3 * sizeof(double),
                           sizeof(double), (size_t)p->S, hipMemcpyDeviceToHost, st));
  QEW_HIP(hipEventRecord(p->rb_event[slot], st));
  p->rb_valid[slot] = true;
  p->rb_next ^= 1;
  return QEW_OK;
}

// Measurement mi of the state in buffer `buf`, from the tile partials already
// written (by the measurement kernels or by a one-step launch that also
// measured): per-sample v, ubar, w2 into the series, and the structure
// factor when the problem asks for it.
qew_status measure_finish(qew_plan_t* p, void* ws, int mi, int buf, hipStream_t st) {
  const Tables t = tables_of(p, ws);
  double* series = series_of(p, ws);
  QEW_HIP(launch_meas_final(t, p->S, partials_of(p, ws), mi, (int)p->meas.size(), series, st));
  if (p->sq_bins > 0) {
    char* b = static_cast<char*>(ws);
    const bool plain = p->precision == QEW_FP64_PLAIN;
    QEW_HIP(launch_sq(t.off, p->S, p->L[0], plain ? plain_buf(p, ws, buf) : nullptr,
                      plain ? SplitBuf{} : split_buf(p, ws, buf),
                      reinterpret_cast<double2*>(b + p->lay.fftA), reinterpret_cast<double2*>(b + p->lay.fftB),
                      reinterpret_cast<const int32_t*>(b + p->lay.sq_chunk_lo),
                      (int)p->sq_chunk_lo.size() - 1, reinterpret_cast<const int32_t*>(b + p->lay.sq_chunk_first),
                      p->sq_bins, reinterpret_cast<double*>(b + p->lay.sq_part),
                      reinterpret_cast<double*>(b + p->lay.sq_series) + (size_t)mi * p->sq_bins, st));
  }
  p->stats.meas_launches++;
  return QEW_OK;
}

// Measurement mi of the current state by the measurement kernels (the split
// state's nodes come from the fused path's cache while it is valid).
qew_status measure(qew_plan_t* p, void* ws, int mi, hipStream_t st) {
  const Tables t = tables_of(p, ws);
  const Phys ph = phys_of(p);
  if (p->precision == QEW_FP64_PLAIN) {
    QEW_HIP(launch_meas_plain(t, plain_buf(p, ws, p->cur_buf), ph, p->kind, partials_of(p, ws), st));
  } else {
    SplitBuf b = split_buf(p, ws, p->cur_buf);
    if (!(fused(p) && p->nodes_valid)) b.nodes = nullptr;
    QEW_HIP(launch_meas_split(t, b, ph, p->kind, partials_of(p, ws), st));
  }
  return measure_finish(p, ws, mi, p->cur_buf, st);
}

qew_status check_ws(const qew_plan_t* p, const void* ws, size_t bytes) {
  if (!p) return fail(QEW_EINVAL, "plan is NULL");
  if (!ws) return fail(QEW_EINVAL, "workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(QEW_EINVAL, "workspace is not 256-byte aligned");
  if (bytes < p->lay.total)
    return fail(QEW_ENOMEM, "workspace holds %zu bytes, the plan needs %zu", bytes, p->lay.total);
  return QEW_OK;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's scratch array (fetched with that
// device current on its first use).
qew_status scratch_of_current_device(char** out) {
  int dev = -1;
  QEW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QEW_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(QEW_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    if ((reinterpret_cast<uintptr_t>(ptr) & 255u) != 0)
      return fail(QEW_EDEVICE, "the scratch array is not 256-byte aligned");
    g_scratch_addr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_addr[dev];
  return QEW_OK;
}

}  // namespace

extern "C" {

const char* qew_last_error(void) { return g_err.c_str(); }

qew_status qew_plan(const qew_problem* pr, qew_plan_t** out) {
  g_err.clear();
  if (!out) return fail(QEW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pr) return fail(QEW_EINVAL, "problem is NULL");
  if (pr->n_samples < 1) return fail(QEW_EINVAL, "n_samples must be >= 1 (got %d)", pr->n_samples);
  if (!pr->L || !pr->f || !pr->disorder_id) return fail(QEW_EINVAL, "L, f and disorder_id must be non-NULL");
  if (pr->kind < QEW_RF_CR_UNIFORM || pr->kind > QEW_RF_PC_GAUSS) return fail(QEW_EINVAL, "unknown disorder kind %d", pr->kind);
  if (pr->period < 0 || pr->period >= (1 << 30)) return fail(QEW_EINVAL, "period must be in [0, 2^30)");
  if (!(std::isfinite(pr->c) && pr->c > 0)) return fail(QEW_EINVAL, "c must be finite and > 0");
  if (!(std::isfinite(pr->dt) && pr->dt > 0)) return fail(QEW_EINVAL, "dt must be finite and > 0");
  if (!(pr->c * pr->dt <= 0.5)) return fail(QEW_EINVAL, "c*dt = %g exceeds 1/2 (explicit Euler is unstable)", pr->c * pr->dt);
  if (!(std::isfinite(pr->strength) && pr->strength >= 0)) return fail(QEW_EINVAL, "strength must be finite and >= 0");
  if (pr->n_steps < 0 || pr->n_steps > (int64_t(1) << 53)) return fail(QEW_EINVAL, "n_steps out of range");
  if (pr->n_meas < 0) return fail(QEW_EINVAL, "n_meas must be >= 0");
  if (pr->n_meas > 0 && !pr->meas_steps) return fail(QEW_EINVAL, "meas_steps is NULL");
  for (int32_t i = 0; i < pr->n_meas; ++i) {
    const int64_t m = pr->meas_steps[i];
    if (m < 0 || m > pr->n_steps) return fail(QEW_EINVAL, "meas_steps[%d] = %lld outside [0, n_steps]", i, (long long)m);
    if (i > 0 && m <= pr->meas_steps[i - 1]) return fail(QEW_EINVAL, "meas_steps must be strictly increasing (index %d)", i);
  }
  if (pr->precision != QEW_FP64_PLAIN && pr->precision != QEW_FP32_SPLIT) return fail(QEW_EINVAL, "unknown precision %d", pr->precision);
  if (pr->path != QEW_ONE_STEP && pr->path != QEW_FUSED) return fail(QEW_EINVAL, "unknown path %d", pr->path);
  if (pr->path == QEW_FUSED && pr->precision != QEW_FP32_SPLIT)
    return fail(QEW_EUNSUPPORTED, "the fused path runs in FP32 split precision only");
  if (pr->k < 0 || pr->k > kMaxHalo) return fail(QEW_EINVAL, "k must be in [0, %d]", kMaxHalo);
  if (pr->tile != 0 && pr->tile != 1024 && pr->tile != 1536 && pr->tile != 2048 && pr->tile != 3072 &&
      pr->tile != 4096)
    return fail(QEW_EINVAL, "tile must be 0, 1024, 1536, 2048, 3072 or 4096");
  if (pr->k > 0 && pr->tile > 0 && 4 * pr->k > pr->tile) return fail(QEW_EINVAL, "need 4*k <= tile");
  if (pr->flags & ~(QEW_FLAG_NO_GRAPH | QEW_FLAG_TIMING | QEW_FLAG_FUSED_DENSE | QEW_FLAG_FUSED_SPARSE))
    return fail(QEW_EINVAL, "unknown flag bits");
  if ((pr->flags & QEW_FLAG_FUSED_DENSE) && (pr->flags & QEW_FLAG_FUSED_SPARSE))
    return fail(QEW_EINVAL, "QEW_FLAG_FUSED_DENSE and QEW_FLAG_FUSED_SPARSE exclude each other");
  if ((pr->flags & (QEW_FLAG_FUSED_DENSE | QEW_FLAG_FUSED_SPARSE)) && pr->path != QEW_FUSED)
    return fail(QEW_EINVAL, "QEW_FLAG_FUSED_DENSE / QEW_FLAG_FUSED_SPARSE apply to the fused path only");
  if (pr->sq_bins < 0) return fail(QEW_EINVAL, "sq_bins must be >= 0");
  if (pr->sq_bins > 0) {
    if (!pr->sq_edges) return fail(QEW_EINVAL, "sq_edges is NULL");
    const int64_t L0 = pr->L[0];
    if (L0 < 8 || L0 > kMaxL || (L0 & (L0 - 1)) != 0)
      return fail(QEW_EINVAL, "the structure factor needs a power-of-two L in [8, 2^30] (got %lld)", (long long)L0);
    for (int32_t s = 1; s < pr->n_samples; ++s)
      if (pr->L[s] != L0) return fail(QEW_EINVAL, "the structure factor needs equal L for every sample");
    if (pr->sq_edges[0] < 1) return fail(QEW_EINVAL, "sq_edges[0] must be >= 1");
    for (int32_t b = 0; b < pr->sq_bins; ++b)
      if (pr->sq_edges[b + 1] <= pr->sq_edges[b]) return fail(QEW_EINVAL, "sq_edges must be strictly increasing (index %d)", b + 1);
    if (pr->sq_edges[pr->sq_bins] > L0 / 2 + 1) return fail(QEW_EINVAL, "sq_edges[%d] exceeds L/2 + 1", pr->sq_bins);
  }
  for (int32_t s = 0; s < pr->n_samples; ++s) {
    if (pr->L[s] < 3 || pr->L[s] > kMaxL) return fail(QEW_EINVAL, "L[%d] = %lld outside [3, 2^30]", s, (long long)pr->L[s]);
    if (!std::isfinite(pr->f[s])) return fail(QEW_EINVAL, "f[%d] is not finite", s);
  }

  qew_plan_t* p = new (std::nothrow) qew_plan_t();
  if (!p) return fail(QEW_EINVAL, "out of host memory");
  p->S = pr->n_samples;
  p->kind = pr->kind;
  p->precision = pr->precision;
  p->path = pr->path;
  p->k_req = pr->k;
  p->tile_req = pr->tile;
  p->flags = pr->flags;
  p->period = pr->period;
  p->sq_bins = pr->sq_bins;
  if (pr->sq_bins > 0) {
    p->sq_edges.assign(pr->sq_edges, pr->sq_edges + pr->sq_bins + 1);
    // Each bin is cut into chunks of at most kSqChunk modes, summed by one
    // workgroup each; a bin then adds its chunks' sums in order.
    for (int32_t b = 0; b < p->sq_bins; ++b) {
      p->sq_chunk_first.push_back((int32_t)p->sq_chunk_lo.size());
      for (int64_t lo = p->sq_edges[b]; lo < p->sq_edges[b + 1]; lo += kSqChunk)
        p->sq_chunk_lo.push_back((int32_t)lo);
    }
    p->sq_chunk_first.push_back((int32_t)p->sq_chunk_lo.size());
    p->sq_chunk_lo.push_back((int32_t)p->sq_edges[p->sq_bins]);
  }
  p->c = pr->c;
  p->dt = pr->dt;
  p->strength = pr->strength;
  p->seed = pr->seed;
  p->n_steps = pr->n_steps;
  p->L.assign(pr->L, pr->L + p->S);
  p->f.assign(pr->f, pr->f + p->S);
  p->did.assign(pr->disorder_id, pr->disorder_id + p->S);
  if (pr->n_meas > 0) p->meas.assign(pr->meas_steps, pr->meas_steps + pr->n_meas);

  int64_t o = 0;
  p->off.resize(p->S);
  p->mt_first.push_back(0);
  for (int32_t s = 0; s < p->S; ++s) {
    p->off[s] = o;
    o += (p->L[s] + 63) / 64 * 64;
    p->total_sites += p->L[s];
    for (int64_t p0 = 0; p0 < p->L[s]; p0 += kMeasTile) {
      p->mt_s.push_back(s);
      p->mt_p0.push_back((int32_t)p0);
      p->mt_len.push_back((int32_t)std::min<int64_t>(kMeasTile, p->L[s] - p0));
    }
    p->mt_first.push_back((int32_t)p->mt_s.size());
  }
  p->padded = o;
  if (p->mt_s.size() > (size_t)INT32_MAX / 2) {
    delete p;
    return fail(QEW_EINVAL, "too many sites");
  }

  if (fused(p)) {
    int64_t cap = 0;
    for (int tile : kTuneTiles) {
      if (p->tile_req && tile != p->tile_req) continue;
      for (int k : kTuneK) {
        const int kk = p->k_req ? p->k_req : k;
        if (4 * kk > tile) continue;
        cap = std::max(cap, fused_tile_count(p, tile, kk));
      }
    }
    if (p->k_req && p->tile_req) cap = fused_tile_count(p, p->tile_req, p->k_req);
    if (cap == 0) {
      delete p;
      return fail(QEW_EINVAL, "no fused geometry satisfies 4*k <= tile");
    }
    if (cap > INT32_MAX / 2) {
      delete p;
      return fail(QEW_EINVAL, "too many fused tiles");
    }
    p->ft_capacity = (int32_t)cap;
    const int tile0 = p->tile_req ? p->tile_req : 2048;
    int k0 = p->k_req ? p->k_req : 16;
    if (4 * k0 > tile0) k0 = tile0 / 4;
    build_fused_tiles(p, tile0, k0);
  } else {
    p->k = 1;
    p->tile = 0;
  }
  compute_layout(p);
  refresh_table_image(p);
  *out = p;
  return QEW_OK;
}

size_t qew_workspace_bytes(const qew_plan_t* p) { return p ? p->lay.total : 0; }

qew_status qew_plan_info_get(const qew_plan_t* p, qew_plan_info* info) {
  if (!p || !info) return fail(QEW_EINVAL, "plan and info must be non-NULL");
  info->total_sites = p->total_sites;
  info->padded_sites = p->padded;
  info->n_tiles = fused(p) ? (int32_t)p->ft_s.size() : (int32_t)p->mt_s.size();
  info->n_meas_tiles = (int32_t)p->mt_s.size();
  info->k = p->k;
  info->tile = p->tile;
  info->autotuned = p->autotuned;
  info->pad_ = 0;
  info->cur_step = p->cur_step;
  return QEW_OK;
}

qew_status qew_run_stats_get(const qew_plan_t* p, qew_run_stats* st) {
  if (!p || !st) return fail(QEW_EINVAL, "plan and stats must be non-NULL");
  *st = p->stats;
  return QEW_OK;
}

qew_status qew_autotune(qew_plan_t* p, void* ws, size_t bytes, void* stream) {
  qew_status rc = check_ws(p, ws, bytes);
  if (rc != QEW_OK) return rc;
  if (!fused(p)) return QEW_OK;
  p->sparse = (p->flags & QEW_FLAG_FUSED_SPARSE) ? 1 : 0;  // time the variant runs start with
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QEW_HIP(hipEventCreate(&e0));
  QEW_HIP(hipEventCreate(&e1));
  double best = -1.0;
  int best_tile = p->tile, best_k = p->k;
  for (int tile : kTuneTiles) {
    if (p->tile_req && tile != p->tile_req) continue;
    if (!fused_fits(tile)) continue;
    for (int kc : kTuneK) {
      const int k = p->k_req ? p->k_req : kc;
      if (4 * k > tile) continue;
      if (p->k_req && kc != kTuneK[0]) continue;  // a fixed k is timed once per tile
      build_fused_tiles(p, tile, k);
      if ((rc = upload_tables(p, ws, st)) != QEW_OK) break;
      if ((rc = init_state(p, ws, st)) != QEW_OK) break;
      if ((rc = ensure_fused_grid(p)) != QEW_OK) break;
      const int steps = std::max(2 * k, 64);
      const int launches = steps / k;
      hipError_t he = step_launch(p, ws, 0, k, st);  // warm-up
      if (he == hipSuccess) he = hipEventRecord(e0, st);
      for (int i = 0; i < launches && he == hipSuccess; ++i) he = step_launch(p, ws, (i + 1) & 1, k, st);
      if (he == hipSuccess) he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) {
        rc = fail(QEW_EDEVICE, "autotune run failed: %s", hipGetErrorString(he));
        break;
      }
      const double rate = (double)p->total_sites * launches * k / (ms > 0 ? ms : 1e-9);
      if (rate > best) {
        best = rate;
        best_tile = tile;
        best_k = k;
      }
    }
    if (rc != QEW_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != QEW_OK) return rc;
  if (best < 0.0) return fail(QEW_EUNSUPPORTED, "no fused tile width fits this device's LDS");
  build_fused_tiles(p, best_tile, best_k);
  p->autotuned = 1;
  p->state_ws = nullptr;  // the state was overwritten
  drop_graphs(p);  // the candidates' launches above have completed (event synchronized)
  return QEW_OK;
}

// qew_run and qew_run_noalloc.  `noalloc`: the small regions (tables,
// partials, series) live in the scratch array at `scratch` and the run makes
// no allocation of any kind: no autotuning, graphs, events, pinned readbacks
// or host buffers; the fused kernel runs its dense variant (or the forced
// one), which gives the same results as the automatic choice.
static qew_status run_impl(qew_plan_t* p, void* ws, size_t bytes, hipStream_t st, int32_t resume,
                           double* h_v, double* h_w2, double* h_ubar, char* scratch) {
  const bool noalloc = scratch != nullptr;
  qew_status rc = check_ws(p, ws, bytes);
  if (rc != QEW_OK) return rc;
  if (resume && (p->state_ws != ws)) return fail(QEW_EINVAL, "resume: this workspace holds no state of this plan");
  if (resume && p->cur_step > p->n_steps) return fail(QEW_EINVAL, "resume: state step beyond n_steps");
  // every run starts dense (or as forced); the variant follows the line from there
  p->sparse = (p->flags & QEW_FLAG_FUSED_SPARSE) ? 1 : 0;
  if (fused(p) && (p->k_req == 0 || p->tile_req == 0) && !p->autotuned) {
    if (resume) return fail(QEW_EINVAL, "resume: run qew_autotune before writing the state");
    if ((rc = qew_autotune(p, ws, bytes, st)) != QEW_OK) return rc;
  }
  // Small regions in the scratch array for this run only (every exit below
  // passes through the guard, which restores the workspace as their base).
  struct SmallBase {
    qew_plan_t* p;
    ~SmallBase() {
      p->small_base = nullptr;
      p->direct_only = false;
    }
  } guard{p};
  p->small_base = scratch;
  p->direct_only = noalloc;
  p->stats = qew_run_stats{};
  if ((rc = upload_tables(p, ws, st)) != QEW_OK) return rc;
  QEW_HIP(launch_fill_i32(tables_of(p, ws).err, 1, 0, st));
  if (noalloc && resume)  // this plan's series so far, from the workspace
    QEW_HIP(hipMemcpyAsync(series_of(p, ws), static_cast<char*>(ws) + p->lay.series,
                           (size_t)p->S * p->meas.size() * 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (fused(p) && !noalloc) {
    if (!p->rb_host)
      QEW_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->rb_host), 2 * (size_t)p->S * sizeof(double)));
    for (int i = 0; i < 2; ++i) {
      if (!p->rb_event[i]) QEW_HIP(hipEventCreateWithFlags(&p->rb_event[i], hipEventDisableTiming));
      p->rb_valid[i] = false;
    }
    p->rb_next = 0;
  }
  if ((rc = ensure_fused_grid(p)) != QEW_OK) return rc;
  if (!resume) {
    if ((rc = init_state(p, ws, st)) != QEW_OK) return rc;
  }
  const bool timing = (p->flags & QEW_FLAG_TIMING) != 0 && !noalloc;
  std::vector<EventPair> step_ev, meas_ev;
  std::vector<char> step_fused;  // per stepping segment: made of fused launches
  EventPair whole;
  auto mk = [&](EventPair& e) -> hipError_t {
    hipError_t r = hipEventCreate(&e.a);
    if (r == hipSuccess) r = hipEventCreate(&e.b);
    return r;
  };
  auto cleanup = [&]() {
    for (auto& e : step_ev) { if (e.a) (void)hipEventDestroy(e.a); if (e.b) (void)hipEventDestroy(e.b); }
    for (auto& e : meas_ev) { if (e.a) (void)hipEventDestroy(e.a); if (e.b) (void)hipEventDestroy(e.b); }
    if (whole.a) (void)hipEventDestroy(whole.a);
    if (whole.b) (void)hipEventDestroy(whole.b);
  };
  // Events around a stepping segment (a stretch's launches of one kind) or a
  // measurement, when timing.
  auto open_ev = [&](std::vector<EventPair>& v) -> hipError_t {
    if (!timing) return hipSuccess;
    v.emplace_back();
    hipError_t r = mk(v.back());
    return r == hipSuccess ? hipEventRecord(v.back().a, st) : r;
  };
  auto close_ev = [&](std::vector<EventPair>& v) -> hipError_t {
    return timing ? hipEventRecord(v.back().b, st) : hipSuccess;
  };
  auto open_step = [&](bool fk) -> hipError_t {
    if (timing) step_fused.push_back(fk ? 1 : 0);
    return open_ev(step_ev);
  };
  const int64_t step0 = p->cur_step;
  const int n_meas = (int)p->meas.size();
  int mi = (int)(std::lower_bound(p->meas.begin(), p->meas.end(), step0) - p->meas.begin());
  const int mi0 = mi;
  hipError_t he = hipSuccess;
  if (timing) {
    he = mk(whole);
    if (he == hipSuccess) he = hipEventRecord(whole.a, st);
  }
  // Walk the stretches between measurement steps.  A stretch that starts at a
  // measurement and runs on the one-step kernel takes that measurement in its
  // first launch; otherwise the measurement kernels run first.  On the fused
  // path, stretches shorter than kShortStretch run on the one-step kernel.
  int64_t m = step0;
  while (he == hipSuccess && rc == QEW_OK) {
    const bool meas_here = mi < n_meas && p->meas[mi] == m;
    if (m >= p->n_steps) {
      if (meas_here) {
        if ((he = open_ev(meas_ev)) != hipSuccess) break;
        if ((rc = measure(p, ws, mi, st)) != QEW_OK) break;
        if ((he = close_ev(meas_ev)) != hipSuccess) break;
        ++mi;
      }
      break;
    }
    const int next = mi + (meas_here ? 1 : 0);
    const int64_t stop = next < n_meas ? p->meas[next] : p->n_steps;
    int64_t n = stop - m;
    const bool onestep = !fused(p) || n < kShortStretch;
    if (meas_here) {
      if (onestep) {
        const int from = p->cur_buf;
        if ((he = open_step(false)) != hipSuccess) break;
        if ((rc = advance_onestep(p, ws, 1, partials_of(p, ws), st)) != QEW_OK) break;
        if ((he = close_ev(step_ev)) != hipSuccess) break;
        if ((he = open_ev(meas_ev)) != hipSuccess) break;
        if ((rc = measure_finish(p, ws, mi, from, st)) != QEW_OK) break;
        if ((he = close_ev(meas_ev)) != hipSuccess) break;
        --n;
      } else {
        if ((he = open_ev(meas_ev)) != hipSuccess) break;
        if ((rc = measure(p, ws, mi, st)) != QEW_OK) break;
        if ((he = close_ev(meas_ev)) != hipSuccess) break;
      }
      if (fused(p) && !noalloc && (rc = post_velocities(p, ws, mi, st)) != QEW_OK) break;
      ++mi;
    }
    if (n > 0 && onestep) {
      if ((he = open_step(false)) != hipSuccess) break;
      if (fused(p)) rc = advance_onestep(p, ws, n, nullptr, st);
      else rc = advance(p, ws, n, st);
      if (rc != QEW_OK) break;
      if ((he = close_ev(step_ev)) != hipSuccess) break;
    } else if (n > 0) {
      if (!p->nodes_valid) {  // after one-step stretches or a written state
        if ((he = open_step(false)) != hipSuccess) break;
        if ((he = launch_refresh_nodes(tables_of(p, ws), split_buf(p, ws, p->cur_buf), phys_of(p), p->kind,
                                       st)) != hipSuccess)
          break;
        if ((he = close_ev(step_ev)) != hipSuccess) break;
        p->nodes_valid = true;
        p->stats.node_refreshes++;
      }
      if (!noalloc && (rc = choose_variant(p)) != QEW_OK) break;
      if ((he = open_step(true)) != hipSuccess) break;
      if ((rc = advance(p, ws, n, st)) != QEW_OK) break;
      if ((he = close_ev(step_ev)) != hipSuccess) break;
    }
    m = stop;
  }
  if (he == hipSuccess && rc == QEW_OK && timing) he = hipEventRecord(whole.b, st);
  if (he != hipSuccess && rc == QEW_OK) rc = fail(QEW_EDEVICE, "event/launch failed: %s", hipGetErrorString(he));
  if (rc != QEW_OK) {
    (void)hipStreamSynchronize(st);
    cleanup();
    p->state_ws = nullptr;
    return rc;
  }
  std::vector<double> series;
  int err_flags = 0;
  const double* d_series = series_of(p, ws);
  if (noalloc) {
    // Each output straight from the device series (rows of {v, ubar, w2} per
    // sample and measurement), then the series back to the workspace so the
    // plan's other calls see this run.
    double* const outs[3] = {h_v, h_ubar, h_w2};
    for (int q = 0; q < 3 && he == hipSuccess && n_meas > mi0; ++q) {
      if (!outs[q]) continue;
      if (mi0 == 0) {
        he = hipMemcpy2DAsync(outs[q], sizeof(double), d_series + q, 3 * sizeof(double), sizeof(double),
                              (size_t)p->S * n_meas, hipMemcpyDeviceToHost, st);
      } else {
        for (int s = 0; s < p->S && he == hipSuccess; ++s)
          he = hipMemcpy2DAsync(outs[q] + (size_t)s * n_meas + mi0, sizeof(double),
                                d_series + ((size_t)s * n_meas + mi0) * 3 + q, 3 * sizeof(double), sizeof(double),
                                (size_t)(n_meas - mi0), hipMemcpyDeviceToHost, st);
      }
    }
    if (he == hipSuccess && n_meas > 0)
      he = hipMemcpyAsync(static_cast<char*>(ws) + p->lay.series, d_series, (size_t)p->S * n_meas * 3 * sizeof(double),
                          hipMemcpyDeviceToDevice, st);
  } else if (n_meas > mi0) {
    series.resize((size_t)p->S * n_meas * 3);
    he = hipMemcpyAsync(series.data(), d_series, series.size() * 8, hipMemcpyDeviceToHost, st);
  }
  if (he == hipSuccess)
    he = hipMemcpyAsync(&err_flags, small_of(p, ws) + p->lay.err, 4, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    cleanup();
    p->state_ws = nullptr;
    return fail(QEW_EDEVICE, "run failed: %s", hipGetErrorString(he));
  }
  if (err_flags) {
    cleanup();
    p->state_ws = nullptr;
    return fail(QEW_EUNSUPPORTED,
                "the cells of a fused tile spread over 2^23 or more (state far from a line); "
                "use the one-step path for this state");
  }
  for (int s = 0; s < p->S && n_meas > mi0 && !noalloc; ++s) {
    for (int i = mi0; i < n_meas; ++i) {
      const double* x = &series[((size_t)s * n_meas + i) * 3];
      if (h_v) h_v[(size_t)s * n_meas + i] = x[0];
      if (h_ubar) h_ubar[(size_t)s * n_meas + i] = x[1];
      if (h_w2) h_w2[(size_t)s * n_meas + i] = x[2];
    }
  }
  if (timing) {
    float ms = 0.0f;
    for (size_t i = 0; i < step_ev.size(); ++i) {
      const EventPair& e = step_ev[i];
      if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) continue;
      p->stats.step_ms += ms;
      if (step_fused[i]) p->stats.fused_ms += ms;
    }
    for (auto& e : meas_ev)
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) p->stats.meas_ms += ms;
    if (hipEventElapsedTime(&ms, whole.a, whole.b) == hipSuccess) p->stats.total_ms = ms;
  }
  cleanup();
  p->stats.site_updates = p->total_sites * (p->n_steps - step0);
  p->cur_step = p->n_steps;
  p->state_ws = ws;
  return QEW_OK;
}

qew_status qew_run(qew_plan_t* p, void* ws, size_t bytes, void* stream, int32_t resume, double* h_v,
                   double* h_w2, double* h_ubar) {
  g_err.clear();
  return run_impl(p, ws, bytes, static_cast<hipStream_t>(stream), resume, h_v, h_w2, h_ubar, nullptr);
}

qew_status qew_run_noalloc(qew_plan_t* p, void* ws, size_t bytes, void* stream, int32_t resume,
                           double* h_v, double* h_w2, double* h_ubar) {
  g_err.clear();
  if (!p) return fail(QEW_EINVAL, "plan is NULL");
  if (p->sq_bins > 0)
    return fail(QEW_EUNSUPPORTED, "qew_run_noalloc: the structure factor's FFT buffers are not scratch-sized; "
                                  "use qew_run");
  if (fused(p) && (p->k_req == 0 || p->tile_req == 0) && !p->autotuned)
    return fail(QEW_EINVAL, "qew_run_noalloc needs a fixed fused geometry: give k and tile in the problem, "
                            "or run qew_autotune first");
  if (p->lay.small_end > kScratchBytes)
    return fail(QEW_ENOMEM, "qew_run_noalloc: the plan's tables, partials and series need %zu bytes; the "
                            "scratch array holds %zu",
                p->lay.small_end, kScratchBytes);
  qew_status rc = check_ws(p, ws, bytes);
  if (rc != QEW_OK) return rc;
  char* scratch_base = nullptr;
  if ((rc = scratch_of_current_device(&scratch_base)) != QEW_OK) return rc;
  return run_impl(p, ws, bytes, static_cast<hipStream_t>(stream), resume, h_v, h_w2, h_ubar, scratch_base);
}

qew_status qew_ensemble(const qew_plan_t* p, const void* ws, void* stream, double* h_out) {
  g_err.clear();
  if (!p || !ws || !h_out) return fail(QEW_EINVAL, "plan, workspace and h_out must be non-NULL");
  if (p->state_ws != ws) return fail(QEW_EINVAL, "this workspace holds no run of this plan");
  const int n_meas = (int)p->meas.size();
  if (n_meas == 0) return QEW_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* w = const_cast<void*>(ws);
  double* ens = reinterpret_cast<double*>(static_cast<char*>(w) + p->lay.ens);
  QEW_HIP(launch_ensemble(p->S, n_meas, series_of(p, w), ens, st));
  QEW_HIP(hipMemcpyAsync(h_out, ens, (size_t)7 * n_meas * 8, hipMemcpyDeviceToHost, st));
  QEW_HIP(hipStreamSynchronize(st));
  return QEW_OK;
}

qew_status qew_sq_get(const qew_plan_t* p, const void* ws, void* stream, double* h_sq) {
  g_err.clear();
  if (!p || !ws || !h_sq) return fail(QEW_EINVAL, "plan, workspace and h_sq must be non-NULL");
  if (p->sq_bins <= 0) return fail(QEW_EINVAL, "the problem has no structure factor bins");
  if (p->state_ws != ws) return fail(QEW_EINVAL, "this workspace holds no run of this plan");
  const size_t n = p->meas.size() * (size_t)p->sq_bins;
  if (n == 0) return QEW_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  QEW_HIP(hipMemcpyAsync(h_sq, static_cast<const char*>(ws) + p->lay.sq_series, n * 8, hipMemcpyDeviceToHost, st));
  QEW_HIP(hipStreamSynchronize(st));
  return QEW_OK;
}

qew_status qew_read_state(const qew_plan_t* p, const void* ws, void* stream, int32_t s, double* h_u,
                          int64_t* h_step) {
  g_err.clear();
  if (!p || !ws || !h_u) return fail(QEW_EINVAL, "plan, workspace and h_u must be non-NULL");
  if (s < 0 || s >= p->S) return fail(QEW_EINVAL, "sample %d out of range", s);
  if (p->state_ws != ws) return fail(QEW_EINVAL, "this workspace holds no state of this plan");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t L = p->L[s];
  void* w = const_cast<void*>(ws);
  if (p->precision == QEW_FP64_PLAIN) {
    QEW_HIP(hipMemcpyAsync(h_u, plain_buf(p, w, p->cur_buf) + p->off[s], L * 8, hipMemcpyDeviceToHost, st));
    QEW_HIP(hipStreamSynchronize(st));
  } else {
    std::vector<int32_t> c(L);
    std::vector<float> r(L);
    const SplitBuf b = split_buf(p, w, p->cur_buf);
    QEW_HIP(hipMemcpyAsync(c.data(), b.cell + p->off[s], L * 4, hipMemcpyDeviceToHost, st));
    QEW_HIP(hipMemcpyAsync(r.data(), b.frac + p->off[s], L * 4, hipMemcpyDeviceToHost, st));
    QEW_HIP(hipStreamSynchronize(st));
    for (int64_t j = 0; j < L; ++j) h_u[j] = (double)c[j] + (double)r[j];
  }
  if (h_step) *h_step = p->cur_step;
  return QEW_OK;
}

qew_status qew_write_state(qew_plan_t* p, void* ws, void* stream, int32_t s, const double* h_u,
                           int64_t step) {
  g_err.clear();
  if (!p || !ws || !h_u) return fail(QEW_EINVAL, "plan, workspace and h_u must be non-NULL");
  if (s < 0 || s >= p->S) return fail(QEW_EINVAL, "sample %d out of range", s);
  if (step < 0 || step > p->n_steps) return fail(QEW_EINVAL, "step outside [0, n_steps]");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(QEW_EINVAL, "workspace is not 256-byte aligned");
  const int64_t L = p->L[s];
  for (int64_t j = 0; j < L; ++j)
    if (!std::isfinite(h_u[j]) || std::fabs(h_u[j]) > 1e9) return fail(QEW_EINVAL, "h_u[%lld] not finite or beyond 1e9", (long long)j);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->state_ws != ws) {
    p->cur_buf = 0;
    qew_status rc = clear_series(p, ws, st);
    if (rc != QEW_OK) return rc;
  }
  if (p->precision == QEW_FP64_PLAIN) {
    QEW_HIP(hipMemcpyAsync(plain_buf(p, ws, p->cur_buf) + p->off[s], h_u, L * 8, hipMemcpyHostToDevice, st));
    QEW_HIP(hipStreamSynchronize(st));
  } else {
    std::vector<int32_t> c(L);
    std::vector<float> r(L);
    for (int64_t j = 0; j < L; ++j) {
      const double fl = std::floor(h_u[j]);
      float fr = (float)(h_u[j] - fl);
      int32_t cc = (int32_t)fl;
      if (fr >= 1.0f) {
        fr = 0.0f;
        cc += 1;
      }
      c[j] = cc;
      r[j] = fr;
    }
    const SplitBuf b = split_buf(p, ws, p->cur_buf);
    QEW_HIP(hipMemcpyAsync(b.cell + p->off[s], c.data(), L * 4, hipMemcpyHostToDevice, st));
    QEW_HIP(hipMemcpyAsync(b.frac + p->off[s], r.data(), L * 4, hipMemcpyHostToDevice, st));
    QEW_HIP(hipStreamSynchronize(st));
  }
  p->cur_step = step;
  p->state_ws = ws;
  p->nodes_valid = false;
  return QEW_OK;
}

qew_status qew_debug_philox_fill(const uint32_t* d_ctr, uint64_t seed, uint32_t* d_out, int64_t N,
                                 void* stream) {
  g_err.clear();
  if (N < 0) return fail(QEW_EINVAL, "N < 0");
  if (N > 0 && (!d_ctr || !d_out)) return fail(QEW_EINVAL, "NULL device pointer");
  if (N > (int64_t(1) << 31) * 256) return fail(QEW_EINVAL, "N too large");
  QEW_HIP(launch_philox_fill(d_ctr, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), d_out, N,
                             static_cast<hipStream_t>(stream)));
  return QEW_OK;
}

qew_status qew_debug_force_eval(int32_t kind, double strength, uint64_t seed, int32_t period,
                                int32_t precision, const uint32_t* d_did, const int32_t* d_j,
                                const int32_t* d_cell, const double* d_frac, double* d_out,
                                int64_t N, void* stream) {
  g_err.clear();
  if (kind < QEW_RF_CR_UNIFORM || kind > QEW_RF_PC_GAUSS) return fail(QEW_EINVAL, "unknown kind");
  if (period < 0 || period >= (1 << 30)) return fail(QEW_EINVAL, "bad period");
  if (precision != QEW_FP64_PLAIN && precision != QEW_FP32_SPLIT) return fail(QEW_EINVAL, "unknown precision");
  if (!(std::isfinite(strength) && strength >= 0)) return fail(QEW_EINVAL, "bad strength");
  if (N < 0) return fail(QEW_EINVAL, "N < 0");
  if (N > 0 && (!d_did || !d_j || !d_cell || !d_frac || !d_out)) return fail(QEW_EINVAL, "NULL device pointer");
  if (N > (int64_t(1) << 31) * 256) return fail(QEW_EINVAL, "N too large");
  QEW_HIP(launch_force_eval(kind, strength, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32),
                            period, precision, d_did, d_j, d_cell, d_frac, d_out, N,
                            static_cast<hipStream_t>(stream)));
  return QEW_OK;
}

qew_status qew_critical_force(int32_t kind, double strength, uint64_t seed, int32_t period, double c,
                              int32_t n_samples, int32_t L, const uint32_t* d_did, double f_lo, double f_hi,
                              double tol_f, double tol_force, int64_t max_sweeps, double* d_u, double* d_f,
                              int64_t* d_status, void* stream) {
  g_err.clear();
  if (kind != QEW_RF_CR_UNIFORM && kind != QEW_RB_CR_GAUSS)
    return fail(QEW_EUNSUPPORTED, "the critical force needs a Catmull-Rom kind (continuous forces)");
  if (!(std::isfinite(strength) && strength >= 0)) return fail(QEW_EINVAL, "strength must be finite and >= 0");
  if (period < 1 || period >= (1 << 30)) return fail(QEW_EINVAL, "the sample must be periodic in u: 1 <= period < 2^30");
  if (!(std::isfinite(c) && c > 0)) return fail(QEW_EINVAL, "c must be finite and > 0");
  if (n_samples < 1) return fail(QEW_EINVAL, "n_samples must be >= 1");
  if (L < 3 || L > kCritMaxL) return fail(QEW_EINVAL, "L must be in [3, %d]", kCritMaxL);
  if (!(std::isfinite(f_lo) && std::isfinite(f_hi) && f_lo < f_hi)) return fail(QEW_EINVAL, "need finite f_lo < f_hi");
  if (!(tol_f > 0) || !(tol_force > 0)) return fail(QEW_EINVAL, "tol_f and tol_force must be > 0");
  if (max_sweeps < 4) return fail(QEW_EINVAL, "max_sweeps must be >= 4");
  const double rounds = std::ceil(std::log2((f_hi - f_lo) / tol_f)) + 1.0;
  if (!(rounds <= 200.0)) return fail(QEW_EINVAL, "(f_hi - f_lo) / tol_f needs more than 200 bisection rounds");
  if (!d_did || !d_u || !d_f || !d_status) return fail(QEW_EINVAL, "NULL device pointer");
  CritParams q;
  q.L = L;
  q.period = period;
  q.max_rounds = (int)std::max(rounds, 1.0);
  q.k0 = (uint32_t)(seed & 0xffffffffu);
  q.k1 = (uint32_t)(seed >> 32);
  q.c = c;
  q.strength = strength;
  q.f_lo = f_lo;
  q.f_hi = f_hi;
  q.tol_f = tol_f;
  q.tol_force = tol_force;
  q.max_sweeps = max_sweeps;
  QEW_HIP(launch_critical(kind, q, n_samples, d_did, d_u, d_f, d_status, static_cast<hipStream_t>(stream)));
  return QEW_OK;
}

void qew_plan_destroy(qew_plan_t* p) {
  if (!p) return;
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->rb_event) {
    if (!e) continue;
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  if (p->rb_host) (void)hipHostFree(p->rb_host);
  delete p;
}

}  // extern "C"
