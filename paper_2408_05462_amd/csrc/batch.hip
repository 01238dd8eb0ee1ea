// batch.hip -- many fields of uneven sizes through compress -> reconstruct
// -> extract as one captured HIP graph.
//
// The items are spread over B parallel branches (longest-first onto the
// least-loaded branch).  Each branch is a stream forked from the caller's
// stream with an event and joined back with one; an item's stages run in
// order on its branch with the same launch plans and kernels as the
// single-field calls, so its outputs are bit for bit theirs.  Capturing the
// fork/join into one graph turns the batch into a single launch whose
// branches the device overlaps.  The autotuner picks B and the level-0 tile
// shapes by timing replays of the captured graph (switched off, see below);
// chr_batch_tune picks B, the brick size and the tiles by timing eager runs
// and captures once.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "capi_internal.h"

using namespace chr;

namespace {

constexpr int kMaxBranches = 8;
// The replay-timed search re-captures and re-instantiates the graph for every
// candidate.  One GPU run aborted inside it (no fault message; the single
// capture + replay path has never failed); it stays off until that is
// explained.
constexpr bool kAutotuneEnabled = false;

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

struct ItemJobs {
  EncJob enc;
  DecJob dec;
  McJob mc[kMaxIso];
};

// Bytes of an item's classification bit planes (one per isovalue), which the
// level-0 decoder writes and marching cubes reads; they sit at the start of
// the branch's region, before the decode / extract scratch.
size_t bits_bytes(const chr_batch_item &it) {
  const size_t plane = (size_t)it.dims[0] * (size_t)it.dims[1] * (size_t)((it.dims[2] + 63) / 64);
  return align256(8 * plane * (size_t)it.n_iso);
}

// One branch's bytes for an item: compression uses the whole region; then
// the bit planes, followed by the reconstruction's or marching cubes'
// scratch.
size_t item_bytes(size_t we, size_t wd, size_t wm, size_t wb) {
  return align256(std::max(we, wb + std::max(wd, wm)));
}

double item_weight(const chr_batch_item &it) {
  return (double)it.dims[0] * (double)it.dims[1] * (double)it.dims[2] * (2.0 + 0.3 * it.n_iso);
}

}  // namespace

struct chr_batch {
  std::vector<chr_batch_item> items;
  std::vector<Geo> geo;
  std::vector<uint64_t> payload_off;
  size_t ws_branch = 0;     // workspace bytes of one branch
  int max_branches = 1;
  int branches = 1;
  int enc_cpw = 8, dec_cpw = 16;  // the process-wide tiles when created
  float last_ms = 0.f;
  std::vector<hipStream_t> streams;
  hipStream_t origin = nullptr;   // capture origin (the caller's stream may be the null stream)
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t exec = nullptr;
  std::vector<int> block0;        // each item's block size as created
};

namespace {

int ensure_streams(chr_batch *b) {
  if (!b->streams.empty()) return CHR_OK;
  b->streams.assign(b->max_branches, nullptr);
  b->join.assign(b->max_branches, nullptr);
  for (int j = 0; j < b->max_branches; j++) {
    if (hipStreamCreateWithFlags(&b->streams[j], hipStreamNonBlocking) != hipSuccess)
      return api_fail(CHR_E_HIP, "hipStreamCreateWithFlags failed");
    if (hipEventCreateWithFlags(&b->join[j], hipEventDisableTiming) != hipSuccess)
      return api_fail(CHR_E_HIP, "hipEventCreateWithFlags failed");
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    return api_fail(CHR_E_HIP, "hipEventCreateWithFlags failed");
  if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess)
    return api_fail(CHR_E_HIP, "hipStreamCreateWithFlags failed");
  return CHR_OK;
}

// Branch of every item for the current branch count: longest first onto the
// least-loaded branch.
std::vector<int> assign(const chr_batch *b) {
  const int n = (int)b->items.size();
  std::vector<int> order(n), br(n, 0);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return item_weight(b->items[x]) > item_weight(b->items[y]); });
  std::vector<double> load(b->branches, 0.0);
  for (int i : order) {
    int best = 0;
    for (int j = 1; j < b->branches; j++)
      if (load[j] < load[best]) best = j;
    br[i] = best;
    load[best] += item_weight(b->items[i]);
  }
  return br;
}

// Host planning of every launch; nothing is enqueued, so a failure here
// leaves no half-issued batch (and no half-captured graph).
int plan(const chr_batch *b, void *d_ws, size_t ws_bytes, std::vector<ItemJobs> &jobs, std::vector<int> &br) {
  if (!d_ws) return api_fail(CHR_E_INVAL, "NULL workspace");
  const size_t need = b->ws_branch * (size_t)b->branches;
  if (ws_bytes < need) return api_fail(CHR_E_NOMEM, "batch workspace too small: need " + std::to_string(need));
  br = assign(b);
  jobs.resize(b->items.size());
  for (size_t i = 0; i < b->items.size(); i++) {
    const chr_batch_item &it = b->items[i];
    uint8_t *ws = static_cast<uint8_t *>(d_ws) + b->ws_branch * (size_t)br[i];
    int rc = enc_prepare(it.d_field, it.dims, it.error_bound, it.isovalues, it.n_iso, &it.params, it.d_stream,
                         it.stream_capacity, it.d_result, nullptr, nullptr, ws, b->ws_branch, b->enc_cpw, jobs[i].enc);
    if (rc) return rc;
    const size_t wb = it.n_iso > 0 ? bits_bytes(it) : 0;
    unsigned long long *bits = reinterpret_cast<unsigned long long *>(ws);
    rc = dec_prepare(b->geo[i], b->payload_off[i], 0, it.d_stream, it.stream_capacity, it.d_recon, it.d_status,
                     ws + wb, b->ws_branch - wb, b->dec_cpw, jobs[i].dec);
    if (rc) return rc;
    const int64_t plane = it.dims[0] * it.dims[1] * ((it.dims[2] + 63) / 64);
    if (it.n_iso > 0) {
      // the level-0 decoder writes the bits of every isovalue
      DecPlan &D = jobs[i].dec.D;
      D.bits = bits;
      D.bnw = (it.dims[2] + 63) / 64;
      D.bplane = plane;
      D.nk = it.n_iso;
      for (int j = 0; j < it.n_iso; j++) D.kb[j] = it.isovalues[j];
    }
    for (int j = 0; j < it.n_iso; j++) {
      rc = mc_prepare(it.d_recon, it.dims, it.isovalues[j], it.spacing, it.d_vertices[j], it.cap_v[j], it.d_tris[j],
                      it.cap_t[j], it.d_counts + 2 * j, ws + wb, b->ws_branch - wb, jobs[i].mc[j]);
      if (rc) return rc;
      jobs[i].mc[j].M.bits = bits + (size_t)j * (size_t)plane;
    }
  }
  return CHR_OK;
}

// Enqueues the planned batch: fork from s, each branch's items in order, join
// back into s.  Only kernel launches and event record/wait, so it can be
// captured.
void enqueue(chr_batch *b, const std::vector<ItemJobs> &jobs, const std::vector<int> &br, hipStream_t s) {
  hipEventRecord(b->fork, s);
  for (int j = 0; j < b->branches; j++) hipStreamWaitEvent(b->streams[j], b->fork, 0);
  for (size_t i = 0; i < jobs.size(); i++) {
    hipStream_t bs = b->streams[br[i]];
    const chr_batch_item &it = b->items[i];
    launch_encode(jobs[i].enc.P, 0, jobs[i].enc.scan, jobs[i].enc.scan64, bs);
    if (it.d_status) launch_status_reset(it.d_status, bs);
    launch_decode(jobs[i].dec.D, bs);
    if (it.n_iso > 0 && !decode_tile0_used(jobs[i].dec.D))
      for (int k = 0; k < it.n_iso; k++) launch_mc_bits(jobs[i].mc[k].M, bs);   // another decoder ran
    for (int k = 0; k < it.n_iso; k++) launch_mc_from_bits(jobs[i].mc[k].M, jobs[i].mc[k].scan, bs);
  }
  for (int j = 0; j < b->branches; j++) {
    hipEventRecord(b->join[j], b->streams[j]);
    hipStreamWaitEvent(s, b->join[j], 0);
  }
}

// Captures on the batch's own origin stream; the graph is later launched on
// whatever stream the caller replays it on.
int capture(chr_batch *b, void *d_ws, size_t ws_bytes) {
  int rc = ensure_streams(b);
  if (rc) return rc;
  std::vector<ItemJobs> jobs;
  std::vector<int> br;
  rc = plan(b, d_ws, ws_bytes, jobs, br);
  if (rc) return rc;
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return api_fail(CHR_E_HIP, "hipStreamBeginCapture failed");
  enqueue(b, jobs, br, b->origin);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(b->origin, &graph);
  if (e != hipSuccess || !graph) return api_fail(CHR_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return api_fail(CHR_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return CHR_OK;
}

// Average duration (ms) of `reps` replays after one untimed replay.
int time_replays(chr_batch *b, hipStream_t s, int reps, float &ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return api_fail(CHR_E_HIP, "hipEventCreate failed");
  hipGraphLaunch(b->exec, s);
  hipEventRecord(e0, s);
  for (int r = 0; r < reps; r++) hipGraphLaunch(b->exec, s);
  hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return api_fail(CHR_E_HIP, std::string("replay timing: ") + hipGetErrorString(e));
  ms = t / (float)reps;
  b->last_ms = ms;
  return CHR_OK;
}

// FNV-1a over the batch's shapes and parameters and the device's name:
// the key of a tuning-cache line.
std::string signature(const chr_batch *b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const uint8_t *c = static_cast<const uint8_t *>(p);
    for (size_t i = 0; i < n; i++) { h ^= c[i]; h *= 1099511628211ull; }
  };
  const int n = (int)b->items.size();
  mix(&n, sizeof(n));
  for (const chr_batch_item &it : b->items) {
    mix(it.dims, sizeof(it.dims));
    mix(&it.params, sizeof(it.params));
    mix(&it.n_iso, sizeof(it.n_iso));
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    mix(&prop.multiProcessorCount, sizeof(int));
  }
  char buf[24];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

bool cache_lookup(const char *path, const std::string &sig, int &br, int &ec, int &dc) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char key[64];
  int a, e, d;
  bool found = false;
  while (std::fscanf(f, "%63s %d %d %d", key, &a, &e, &d) == 4)
    if (sig == key && a >= 1 && a <= kMaxBranches && tiles_ok(e, d)) { br = a; ec = e; dc = d; found = true; }
  std::fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &sig, int br, int ec, int dc) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d\n", sig.c_str(), br, ec, dc);
  std::fclose(f);
}

// Workspace bytes of one branch for the items' current parameters (0 when
// some item's parameters are invalid).
size_t branch_bytes(const chr_batch *b, const std::vector<Geo> &geo) {
  size_t ws = 0;
  for (size_t i = 0; i < b->items.size(); i++) {
    const chr_batch_item &it = b->items[i];
    const size_t we = enc_workspace_bytes(it.dims, &it.params);
    const size_t wd = dec_workspace_bytes(geo[i], 0);
    const size_t wm = it.n_iso > 0 ? mc_workspace_bytes(it.dims) : 0;
    if (!we || (it.n_iso > 0 && !wm)) return 0;
    ws = std::max(ws, item_bytes(we, wd, wm, it.n_iso > 0 ? bits_bytes(it) : 0));
  }
  return ws;
}

// Gives every item brick size B (0: each item's own, as created) when it is
// valid for all of them, their streams fit the capacities and one branch's
// workspace times `branches` fits ws_bytes; otherwise nothing changes.
int set_block(chr_batch *b, int B, int branches, size_t ws_bytes) {
  std::vector<chr_batch_item> items = b->items;
  std::vector<Geo> geo(items.size());
  std::vector<uint64_t> poff(items.size());
  for (size_t i = 0; i < items.size(); i++) {
    chr_batch_item &it = items[i];
    it.params.block = B ? B : b->block0[i];
    int rc = enc_geometry(it.dims, it.error_bound, it.isovalues, it.n_iso, &it.params, geo[i], poff[i]);
    if (rc) return rc;
    const size_t need = chr_compress_bound(it.dims, &it.params);
    if (!need || need > it.stream_capacity) return api_fail(CHR_E_CAPACITY, "stream capacity below the bound");
  }
  std::swap(b->items, items);
  const size_t ws = branch_bytes(b, geo);
  if (!ws || ws * (size_t)branches > ws_bytes) {
    std::swap(b->items, items);
    return api_fail(CHR_E_NOMEM, "workspace too small for this block size");
  }
  b->geo = geo;
  b->payload_off = poff;
  b->ws_branch = ws;
  return CHR_OK;
}

// Average duration (ms) of `reps` eager runs on s after one untimed run.
int time_eager(chr_batch *b, void *d_ws, size_t ws_bytes, hipStream_t s, int reps, float &ms) {
  std::vector<ItemJobs> jobs;
  std::vector<int> br;
  int rc = plan(b, d_ws, ws_bytes, jobs, br);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return api_fail(CHR_E_HIP, "hipEventCreate failed");
  }
  enqueue(b, jobs, br, s);
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; r++) {
    enqueue(b, jobs, br, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return api_fail(CHR_E_HIP, std::string("eager timing: ") + hipGetErrorString(e));
  ms = t / (float)reps;
  b->last_ms = ms;
  return CHR_OK;
}

bool cache_lookup5(const char *path, const std::string &sig, int v[4]) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char key[64];
  int a, B, e, d;
  bool found = false;
  while (std::fscanf(f, "%63s %d %d %d %d", key, &a, &B, &e, &d) == 5)
    if (sig == key && a >= 1 && a <= kMaxBranches && B >= 0 && tiles_ok(e, d)) {
      v[0] = a; v[1] = B; v[2] = e; v[3] = d;
      found = true;
    }
  std::fclose(f);
  return found;
}

}  // namespace

extern "C" {

int chr_batch_create(const chr_batch_item *items, int n_items, chr_batch **out) {
  if (!out || !items || n_items < 1) return api_fail(CHR_E_INVAL, "need at least one item and an output pointer");
  *out = nullptr;
  chr_batch *b = new chr_batch;
  current_tiles(b->enc_cpw, b->dec_cpw);
  b->items.assign(items, items + n_items);
  b->geo.resize(n_items);
  b->payload_off.resize(n_items);
  for (int i = 0; i < n_items; i++) {
    const chr_batch_item &it = b->items[i];
    const std::string at = "item " + std::to_string(i) + ": ";
    int rc = enc_geometry(it.dims, it.error_bound, it.isovalues, it.n_iso, &it.params, b->geo[i], b->payload_off[i]);
    if (rc) { delete b; return api_fail(rc, at + chr_last_error()); }
    if (!it.d_field || !it.d_stream || !it.d_result || !it.d_recon || (it.n_iso > 0 && !it.d_counts)) {
      delete b;
      return api_fail(CHR_E_INVAL, at + "NULL device pointer");
    }
    if (it.stream_capacity < b->payload_off[i]) {
      delete b;
      return api_fail(CHR_E_CAPACITY, at + "stream capacity below the header and tables");
    }
    for (int j = 0; j < it.n_iso; j++)
      if (it.cap_v[j] < 0 || it.cap_t[j] < 0 || (it.cap_v[j] && !it.d_vertices[j]) || (it.cap_t[j] && !it.d_tris[j])) {
        delete b;
        return api_fail(CHR_E_INVAL, at + "bad mesh capacity");
      }
    const size_t we = enc_workspace_bytes(it.dims, &it.params);
    const size_t wd = dec_workspace_bytes(b->geo[i], 0);
    const size_t wm = it.n_iso > 0 ? mc_workspace_bytes(it.dims) : 0;
    if (!we || (it.n_iso > 0 && !wm)) { delete b; return api_fail(CHR_E_INVAL, at + chr_last_error()); }
    b->ws_branch = std::max(b->ws_branch, item_bytes(we, wd, wm, it.n_iso > 0 ? bits_bytes(it) : 0));
  }
  for (const chr_batch_item &it : b->items) b->block0.push_back(it.params.block);
  b->max_branches = std::min(kMaxBranches, n_items);
  b->branches = b->max_branches;  // measured: throughput grows up to 8 branches (batch64)
  *out = b;
  return CHR_OK;
}

size_t chr_batch_workspace(const chr_batch *b) { return b ? b->ws_branch * (size_t)b->max_branches : 0; }

int chr_batch_run(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  int rc = ensure_streams(b);
  if (rc) return rc;
  std::vector<ItemJobs> jobs;
  std::vector<int> br;
  rc = plan(b, d_ws, ws_bytes, jobs, br);
  if (rc) return rc;
  enqueue(b, jobs, br, static_cast<hipStream_t>(stream));
  return api_check_launch("chr_batch_run");
}

int chr_batch_capture(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  (void)stream;  // captured on the batch's origin stream; replays choose their stream
  return capture(b, d_ws, ws_bytes);
}

int chr_batch_replay(chr_batch *b, void *stream) {
  if (!b || !b->exec) return api_fail(CHR_E_INVAL, "batch not captured");
  hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return api_fail(CHR_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return CHR_OK;
}

int chr_batch_autotune(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream, const char *cache_path) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  if (!kAutotuneEnabled)
    return api_fail(CHR_E_INVAL, "chr_batch_autotune is switched off: one run aborted inside its capture/replay "
                                 "search on the GPU and the cause is not yet known");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string sig = signature(b);
  int cb, ce, cd;
  if (cache_lookup(cache_path, sig, cb, ce, cd) && cb <= b->max_branches) {
    b->branches = cb;
    b->enc_cpw = ce;
    b->dec_cpw = cd;
    return capture(b, d_ws, ws_bytes);
  }
  const int reps = 3;
  auto measure = [&](int br, int ec, int dc, float &ms) {
    b->branches = br;
    b->enc_cpw = ec;
    b->dec_cpw = dc;
    int rc = capture(b, d_ws, ws_bytes);
    return rc ? rc : time_replays(b, s, reps, ms);
  };
  int best[3] = {b->branches, b->enc_cpw, b->dec_cpw};
  float best_ms = 0.f;
  int rc = measure(best[0], best[1], best[2], best_ms);
  if (rc) return rc;
  const std::vector<int> cand[3] = {{1, 2, 4, 8}, {1, 2, 4, 8}, {8, 16, 32, 64}};
  // coordinate descent: branches, then compression tiles, then reconstruction tiles
  for (int dim = 0; dim < 3; dim++) {
    for (int v : cand[dim]) {
      if (v == best[dim] || (dim == 0 && v > b->max_branches)) continue;
      int c[3] = {best[0], best[1], best[2]};
      c[dim] = v;
      float ms = 0.f;
      rc = measure(c[0], c[1], c[2], ms);
      if (rc) return rc;
      if (ms < 0.99f * best_ms) {
        best_ms = ms;
        std::copy(c, c + 3, best);
      }
    }
  }
  b->branches = best[0];
  b->enc_cpw = best[1];
  b->dec_cpw = best[2];
  rc = capture(b, d_ws, ws_bytes);
  if (rc) return rc;
  b->last_ms = best_ms;
  cache_store(cache_path, sig, best[0], best[1], best[2]);
  return CHR_OK;
}

int chr_batch_tune(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream, const char *cache_path,
                   int *block_out) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  if (!d_ws) return api_fail(CHR_E_INVAL, "NULL workspace");
  int rc = ensure_streams(b);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string sig = "t" + signature(b);
  int cur[4] = {b->branches, 0, b->enc_cpw, b->dec_cpw};   // branches, block (0: as created), tiles
  auto apply = [&](const int c[4]) {
    int r = set_block(b, c[1], c[0], ws_bytes);
    if (r) return r;
    b->branches = c[0];
    b->enc_cpw = c[2];
    b->dec_cpw = c[3];
    return CHR_OK;
  };
  int cached[4];
  if (cache_lookup5(cache_path, sig, cached) && cached[0] <= b->max_branches && apply(cached) == CHR_OK) {
    if (block_out) *block_out = cached[1];
    return capture(b, d_ws, ws_bytes);
  }
  const int reps = 2;
  float best_ms = 0.f;
  rc = apply(cur);
  if (rc) return rc;
  rc = time_eager(b, d_ws, ws_bytes, s, reps, best_ms);
  if (rc) return rc;
  // coordinate descent: brick size, branches, compression tiles,
  // reconstruction tiles; a change is kept when at least 1% faster, and a
  // candidate that does not fit (block size invalid for an item, stream or
  // workspace too small) is skipped
  const std::vector<int> cand[4] = {{1, 2, 4, 8}, {0, 32, 64, 128}, {1, 2, 4, 8, 16}, {8, 16, 32, 64}};
  const int order[4] = {1, 0, 2, 3};
  for (int oi = 0; oi < 4; oi++) {
    const int dim = order[oi];
    for (int v : cand[dim]) {
      if (v == cur[dim] || (dim == 0 && v > b->max_branches)) continue;
      int c[4] = {cur[0], cur[1], cur[2], cur[3]};
      c[dim] = v;
      if (apply(c) != CHR_OK) continue;
      float ms = 0.f;
      rc = time_eager(b, d_ws, ws_bytes, s, reps, ms);
      if (rc) return rc;
      if (ms < 0.99f * best_ms) {
        best_ms = ms;
        std::copy(c, c + 4, cur);
      }
    }
  }
  rc = apply(cur);
  if (rc) return rc;
  rc = capture(b, d_ws, ws_bytes);
  if (rc) return rc;
  b->last_ms = best_ms;
  if (block_out) *block_out = cur[1];
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %d %d %d\n", sig.c_str(), cur[0], cur[1], cur[2], cur[3]);
      std::fclose(f);
    }
  }
  return CHR_OK;
}

int chr_batch_set_config(chr_batch *b, int branches, int enc_cpw, int dec_cpw) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  if (branches < 1 || branches > b->max_branches)
    return api_fail(CHR_E_INVAL, "branches must be 1 .. " + std::to_string(b->max_branches));
  if (!tiles_ok(enc_cpw, dec_cpw))
    return api_fail(CHR_E_INVAL, "tiles: compression 1, 2, 4, 8 or 16; reconstruction 8, 16, 32 or 64 chunks per wave");
  b->branches = branches;
  b->enc_cpw = enc_cpw;
  b->dec_cpw = dec_cpw;
  return CHR_OK;
}

int chr_batch_config(const chr_batch *b, int *branches, int *enc_cpw, int *dec_cpw, float *last_ms) {
  if (!b) return api_fail(CHR_E_INVAL, "NULL batch");
  if (branches) *branches = b->branches;
  if (enc_cpw) *enc_cpw = b->enc_cpw;
  if (dec_cpw) *dec_cpw = b->dec_cpw;
  if (last_ms) *last_ms = b->last_ms;
  return CHR_OK;
}

int chr_batch_destroy(chr_batch *b) {
  if (!b) return CHR_OK;
  if (b->exec) hipGraphExecDestroy(b->exec);
  for (hipStream_t st : b->streams)
    if (st) hipStreamDestroy(st);
  for (hipEvent_t e : b->join)
    if (e) hipEventDestroy(e);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->origin) hipStreamDestroy(b->origin);
  delete b;
  return CHR_OK;
}

}  // extern "C"
