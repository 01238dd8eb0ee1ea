// serve.hip -- request loop over resident CHR streams: FIFO admission by
// memory footprint into slots (HIP streams), groups of requests sharing one
// reconstruction, two-phase marching cubes (count on the device, read the
// counts, allocate exactly, emit).  Host code only; the device work is the
// launch plans of chr_reconstruct and iso_extract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "capi_internal.h"

using namespace chr;

namespace {

constexpr int kMaxSlots = 16;
constexpr int kMaxGroup = 64;
constexpr size_t kAlign = 256;

size_t align_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over byte offsets of the caller's pool.
struct Pool {
  size_t bytes = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> size, coalesced

  void init(size_t n) {
    bytes = n & ~(kAlign - 1);
    free_.clear();
    if (bytes) free_[0] = bytes;
    used = peak = 0;
  }
  bool alloc(size_t n, size_t &off) {
    n = align_up(std::max<size_t>(n, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      off = it->first;
      const size_t rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used += n;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(std::max<size_t>(n, 1));
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Block {
  size_t off = 0, n = 0;
  bool live = false;
};

struct StreamRec {
  int dataset;
  chr_info info;
  Geo g;
  const void *d;
};

enum State { QUEUED, RUNNING, DONE, FAILED, CANCELLED, RELEASED };

// Sizes of marching cubes on a field of dims n.
struct McSizes {
  int64_t nrows, nw, nwords;
  size_t bits, cnt, P, scan, counts, total;  // counting state
};

McSizes mc_sizes(const int64_t n[3]) {
  McSizes z;
  z.nrows = n[0] * n[1];
  z.nw = ceil_div(n[2], 64);
  z.nwords = z.nrows * z.nw;
  z.bits = align_up(8 * (size_t)z.nwords);
  z.cnt = align_up(sizeof(uint32_t) * (size_t)z.nwords);
  z.P = align_up(sizeof(U4) * (size_t)(z.nwords + 1));
  z.scan = align_up(sizeof(U4) * (size_t)scan_tmp_elems(z.nwords));
  z.counts = align_up(4 * sizeof(int64_t));
  z.total = z.bits + z.cnt + z.P + z.scan + z.counts;
  return z;
}

struct Req {
  int64_t id;
  int dataset, sidx, level;
  float k;
  double acc;
  State state = QUEUED;
  int status = CHR_PENDING;
  bool cancelled = false;
  int group_size = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  Block cstate, lists, mesh;
  McPlan M;
  U4 *scan = nullptr;
  int phase = 0;        // 1 counted (waiting for memory), 2 emitting, 3 finished
  int64_t nv = 0, nt = 0, npv = 0, nac = 0;
};

struct Group {
  bool busy = false;
  bool inflight = false;  // device work recorded on the slot's event and not yet seen finished
  int sidx = -1, level = 0;
  int64_t seq = 0;        // admission order
  std::vector<int64_t> reqs;
  Block recon;            // status word, reconstruction, decode workspace
  int stage = 0;          // 1 counting, 2 emitting
  int64_t dims[3];
};

int64_t lvl_n(int64_t n, int l) { return ((n - 1) >> l) + 1; }

}  // namespace

struct chr_server {
  chr_server_config cfg;
  Pool pool;
  std::vector<StreamRec> streams;
  std::vector<Req> reqs;          // index = id
  std::deque<int64_t> queue;
  Group slot[kMaxSlots];
  std::vector<hipStream_t> hs;    // created on the first step
  std::vector<hipEvent_t> ev;
  int64_t *h_pinned = nullptr;    // per slot: [status, pad, pad, pad] + max_group x 4 counts
  std::chrono::steady_clock::time_point t0;
  chr_server_stats st{};
  int64_t seq = 0;
};

namespace {

double now_ms(const chr_server *s) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0).count();
}

uint8_t *pool_ptr(const chr_server *s, size_t off) { return static_cast<uint8_t *>(s->cfg.d_pool) + off; }

size_t slot_pinned_words(const chr_server *s) { return 4 + 4 * (size_t)s->cfg.max_group; }

// Bytes of the group block: status word, reconstruction, decode workspace.
size_t group_bytes(const StreamRec &r, int level) {
  int64_t d[3];
  for (int a = 0; a < 3; a++) d[a] = lvl_n(r.info.dims[a], level);
  return kAlign + align_up(4 * (size_t)(d[0] * d[1] * d[2])) + align_up(dec_workspace_bytes(r.g, level));
}

void free_block(chr_server *s, Block &b) {
  if (b.live) s->pool.release(b.off, b.n);
  b.live = false;
}

bool alloc_block(chr_server *s, Block &b, size_t n) {
  if (!s->pool.alloc(n, b.off)) return false;
  b.n = n;
  b.live = true;
  return true;
}

void finish(chr_server *s, Req &r, int status) {
  r.phase = 3;
  r.t_done = now_ms(s);
  free_block(s, r.cstate);
  free_block(s, r.lists);
  if (r.cancelled) {
    free_block(s, r.mesh);
    r.state = CANCELLED;
    r.status = CHR_E_CANCELLED;
    s->st.failed++;
    return;
  }
  r.status = status;
  if (status == CHR_OK) {
    r.state = DONE;
    s->st.done++;
  } else {
    free_block(s, r.mesh);
    r.state = FAILED;
    s->st.failed++;
  }
}

int ensure_device(chr_server *s) {
  if (!s->hs.empty()) return CHR_OK;
  s->hs.assign(s->cfg.slots, nullptr);
  s->ev.assign(s->cfg.slots, nullptr);
  for (int j = 0; j < s->cfg.slots; j++) {
    if (hipStreamCreateWithFlags(&s->hs[j], hipStreamNonBlocking) != hipSuccess)
      return api_fail(CHR_E_HIP, "hipStreamCreateWithFlags failed");
    if (hipEventCreateWithFlags(&s->ev[j], hipEventDisableTiming) != hipSuccess)
      return api_fail(CHR_E_HIP, "hipEventCreateWithFlags failed");
  }
  const size_t bytes = sizeof(int64_t) * slot_pinned_words(s) * (size_t)s->cfg.slots;
  if (hipHostMalloc(reinterpret_cast<void **>(&s->h_pinned), bytes, hipHostMallocDefault) != hipSuccess)
    return api_fail(CHR_E_HIP, "hipHostMalloc failed");
  std::memset(s->h_pinned, 0, bytes);
  return CHR_OK;
}

// Launches the reconstruction of a new group and the counting half of
// marching cubes of each of its requests, then the copy of the status and
// counts to pinned host memory.
int launch_group(chr_server *s, int j) {
  Group &G = s->slot[j];
  const StreamRec &R = s->streams[G.sidx];
  hipStream_t hs = s->hs[j];
  uint8_t *base = pool_ptr(s, G.recon.off);
  int32_t *status = reinterpret_cast<int32_t *>(base);
  float *recon = reinterpret_cast<float *>(base + kAlign);
  const size_t rbytes = align_up(4 * (size_t)(G.dims[0] * G.dims[1] * G.dims[2]));
  uint8_t *dws = base + kAlign + rbytes;
  DecJob dj;
  const int rc = dec_prepare(R.g, R.info.payload_offset, G.level, R.d, R.info.total_bytes, recon, status, dws,
                             dec_workspace_bytes(R.g, G.level), 16, dj);
  if (rc) return rc;
  // only the blocks the group's isovalues need are reconstructed
  float kmin = s->reqs[G.reqs[0]].k, kmax = kmin;
  for (int64_t id : G.reqs) {
    kmin = std::min(kmin, s->reqs[id].k);
    kmax = std::max(kmax, s->reqs[id].k);
  }
  dj.D.prune = 1;
  dj.D.kmin = kmin;
  dj.D.kmax = kmax;
  launch_status_reset(status, hs);
  launch_decode(dj.D, hs);
  int64_t *pin = s->h_pinned + slot_pinned_words(s) * j;
  hipMemcpyAsync(pin, status, sizeof(int32_t), hipMemcpyDeviceToHost, hs);
  const McSizes z = mc_sizes(G.dims);
  for (size_t q = 0; q < G.reqs.size(); q++) {
    Req &r = s->reqs[G.reqs[q]];
    uint8_t *c = pool_ptr(s, r.cstate.off);
    McPlan &M = r.M;
    std::memset(&M, 0, sizeof(M));
    for (int a = 0; a < 3; a++) M.n[a] = G.dims[a];
    M.nrows = z.nrows;
    M.nw = z.nw;
    M.f = recon;
    M.py = G.dims[2];
    M.pz = G.dims[1] * G.dims[2];
    M.k = r.k;
    M.spacing = (float)(1 << r.level);
    M.bits = reinterpret_cast<unsigned long long *>(c);
    M.cnt = reinterpret_cast<uint32_t *>(c + z.bits);
    M.P = reinterpret_cast<U4 *>(c + z.bits + z.cnt);
    r.scan = reinterpret_cast<U4 *>(c + z.bits + z.cnt + z.P);
    M.counts = reinterpret_cast<int64_t *>(c + z.bits + z.cnt + z.P + z.scan);
    launch_mc_count(M, r.scan, hs);
    hipMemcpyAsync(pin + 4 + 4 * q, M.counts, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, hs);
  }
  hipEventRecord(s->ev[j], hs);
  G.stage = 1;
  G.inflight = true;
  return CHR_OK;
}

size_t list_bytes(const Req &r) {
  return align_up(4 * (size_t)r.npv) + align_up(4 * (size_t)r.nac) + align_up(4 * (size_t)(r.nac / 256 + 1));
}
size_t mesh_bytes(const Req &r) { return align_up(12 * (size_t)r.nv) + align_up(12 * (size_t)r.nt); }

// Emitting half for the counted requests of slot j, in order, as far as the
// pool holds their lists and meshes.  Returns how many were launched.
int launch_emits(chr_server *s, int j) {
  Group &G = s->slot[j];
  hipStream_t hs = s->hs[j];
  int launched = 0;
  for (int64_t id : G.reqs) {
    Req &r = s->reqs[id];
    if (r.phase != 1) continue;
    if (r.cancelled) {
      finish(s, r, CHR_E_CANCELLED);
      continue;
    }
    if (!alloc_block(s, r.lists, list_bytes(r))) break;
    if (!alloc_block(s, r.mesh, mesh_bytes(r))) {
      free_block(s, r.lists);
      break;
    }
    McPlan &M = r.M;
    uint8_t *l = pool_ptr(s, r.lists.off);
    M.vlist = reinterpret_cast<uint32_t *>(l);
    M.clist = reinterpret_cast<uint32_t *>(l + align_up(4 * (size_t)r.npv));
    M.tb = reinterpret_cast<uint32_t *>(l + align_up(4 * (size_t)r.npv) + align_up(4 * (size_t)r.nac));
    M.cap_pv = r.npv;
    M.cap_ac = r.nac;
    uint8_t *m = pool_ptr(s, r.mesh.off);
    M.verts = reinterpret_cast<float *>(m);
    M.tris = reinterpret_cast<int32_t *>(m + align_up(12 * (size_t)r.nv));
    M.cap_v = r.nv;
    M.cap_t = r.nt;
    launch_mc_emit(M, hs);
    r.phase = 2;
    launched++;
  }
  if (launched) {
    hipEventRecord(s->ev[j], hs);
    G.inflight = true;
  }
  return launched;
}

bool group_finished(const chr_server *s, const Group &G) {
  for (int64_t id : G.reqs)
    if (s->reqs[id].phase != 3) return false;
  return true;
}

void close_group(chr_server *s, int j) {
  Group &G = s->slot[j];
  free_block(s, G.recon);
  G.reqs.clear();
  G.busy = false;
  G.inflight = false;
  G.stage = 0;
}

// Puts the waiting requests of slot j back at the head of the queue (their
// counting is redone later) and frees what they held.
void preempt(chr_server *s, int j) {
  Group &G = s->slot[j];
  std::vector<int64_t> back;
  for (int64_t id : G.reqs) {
    Req &r = s->reqs[id];
    if (r.phase != 1) continue;
    free_block(s, r.cstate);
    r.phase = 0;
    r.state = QUEUED;
    r.group_size = 0;
    back.push_back(id);
  }
  s->queue.insert(s->queue.begin(), back.begin(), back.end());
  std::sort(s->queue.begin(), s->queue.end());
  close_group(s, j);
}

// Admits the head of the queue (and the queued requests sharing its stream
// and level, up to max_group and what the pool holds) into slot j.
bool admit(chr_server *s, int j) {
  while (!s->queue.empty() && s->reqs[s->queue.front()].state != QUEUED) s->queue.pop_front();
  if (s->queue.empty()) return false;
  Req &head = s->reqs[s->queue.front()];
  Group &G = s->slot[j];
  const StreamRec &R = s->streams[head.sidx];
  for (int a = 0; a < 3; a++) G.dims[a] = lvl_n(R.info.dims[a], head.level);
  if (!alloc_block(s, G.recon, group_bytes(R, head.level))) return false;
  const McSizes z = mc_sizes(G.dims);
  G.sidx = head.sidx;
  G.level = head.level;
  G.reqs.clear();
  std::deque<int64_t> rest;
  for (int64_t id : s->queue) {
    Req &r = s->reqs[id];
    if (r.state != QUEUED) continue;
    if ((int)G.reqs.size() < s->cfg.max_group && r.sidx == G.sidx && r.level == G.level &&
        alloc_block(s, r.cstate, z.total)) {
      G.reqs.push_back(id);
    } else {
      rest.push_back(id);
    }
  }
  if (G.reqs.empty()) {  // not even the head's counting state fits
    free_block(s, G.recon);
    return false;
  }
  s->queue.swap(rest);
  const double t = now_ms(s);
  for (int64_t id : G.reqs) {
    Req &r = s->reqs[id];
    r.state = RUNNING;
    r.t_admit = t;
    r.group_size = (int)G.reqs.size();
  }
  s->st.groups++;
  s->st.grouped_requests += (int64_t)G.reqs.size();
  G.busy = true;
  G.seq = s->seq++;
  if (launch_group(s, j) != CHR_OK) {  // nothing was launched
    for (int64_t id : G.reqs) finish(s, s->reqs[id], CHR_E_INVAL);
    close_group(s, j);
  }
  return true;
}

}  // namespace

extern "C" {

int chr_server_create(const chr_server_config *cfg, chr_server **out) {
  if (!cfg || !out) return api_fail(CHR_E_INVAL, "NULL argument");
  if (cfg->slots < 1 || cfg->slots > kMaxSlots) return api_fail(CHR_E_INVAL, "slots must be in [1, 16]");
  if (cfg->max_group < 1 || cfg->max_group > kMaxGroup) return api_fail(CHR_E_INVAL, "max_group must be in [1, 64]");
  if (!cfg->d_pool || cfg->pool_bytes < kAlign) return api_fail(CHR_E_INVAL, "pool missing or too small");
  chr_server *s = new chr_server;
  s->cfg = *cfg;
  s->pool.init(cfg->pool_bytes);
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return CHR_OK;
}

int chr_server_add_stream(chr_server *s, int dataset, const chr_info *info, const void *d_stream, size_t stream_bytes,
                          int *index) {
  if (!s || !info || !d_stream) return api_fail(CHR_E_INVAL, "NULL argument");
  StreamRec r;
  r.dataset = dataset;
  r.info = *info;
  r.d = d_stream;
  int rc = info_geo(info, r.g);
  if (rc) return rc;
  if (stream_bytes < info->total_bytes) return api_fail(CHR_E_CORRUPT, "stream shorter than its header states");
  if (r.g.nblocks > 65535) return api_fail(CHR_E_INVAL, "more than 65535 blocks");
  s->streams.push_back(r);
  if (index) *index = (int)s->streams.size() - 1;
  return CHR_OK;
}

int chr_server_submit(chr_server *s, int dataset, float isovalue, double accuracy, int level, int64_t *id) {
  if (!s || !id) return api_fail(CHR_E_INVAL, "NULL argument");
  if (!std::isfinite(isovalue)) return api_fail(CHR_E_INVAL, "isovalue must be finite");
  int best = -1;
  bool known = false;
  for (size_t i = 0; i < s->streams.size(); i++) {
    const StreamRec &r = s->streams[i];
    if (r.dataset != dataset) continue;
    known = true;
    if (stream_bound(r.info) <= accuracy && (best < 0 || stream_bound(r.info) > stream_bound(s->streams[best].info)))
      best = (int)i;
  }
  if (!known) return api_fail(CHR_E_INVAL, "unknown dataset");
  if (best < 0) return api_fail(CHR_E_ACCURACY, "no stream of the dataset meets the accuracy");
  const StreamRec &R = s->streams[best];
  if (level < 0 || level >= R.info.levels) return api_fail(CHR_E_LEVEL, "level outside the hierarchy");
  int64_t d[3];
  for (int a = 0; a < 3; a++) d[a] = lvl_n(R.info.dims[a], level);
  if ((double)d[0] * (double)d[1] * (double)ceil_div(d[2], 64) * 64.0 >= 4294967296.0)
    return api_fail(CHR_E_INVAL, "level too large for marching cubes (2^32 padded points)");
  const size_t need = align_up(group_bytes(R, level)) + align_up(mc_sizes(d).total);
  if (need > s->pool.bytes) return api_fail(CHR_E_NOMEM, "request footprint " + std::to_string(need) + " exceeds the pool");
  Req r;
  r.id = (int64_t)s->reqs.size();
  r.dataset = dataset;
  r.sidx = best;
  r.level = level;
  r.k = isovalue;
  r.acc = accuracy;
  r.t_submit = now_ms(s);
  std::memset(&r.M, 0, sizeof(r.M));
  s->reqs.push_back(r);
  s->queue.push_back(r.id);
  *id = r.id;
  return CHR_OK;
}

int chr_server_step(chr_server *s, int *n_done) {
  if (!s) return api_fail(CHR_E_INVAL, "NULL server");
  if (n_done) *n_done = 0;
  int rc = ensure_device(s);
  if (rc) return rc;
  const int64_t done0 = s->st.done + s->st.failed;
  for (int j = 0; j < s->cfg.slots; j++) {
    Group &G = s->slot[j];
    if (!G.busy) continue;
    if (G.inflight) {
      const hipError_t q = hipEventQuery(s->ev[j]);
      if (q == hipErrorNotReady) continue;
      G.inflight = false;
      if (q != hipSuccess) {
        for (int64_t id : G.reqs)
          if (s->reqs[id].phase != 3) finish(s, s->reqs[id], CHR_E_HIP);
        close_group(s, j);
        api_fail(CHR_E_HIP, std::string("device work of a group failed: ") + hipGetErrorString(q));
        continue;
      }
      const int64_t *pin = s->h_pinned + slot_pinned_words(s) * j;
      if (G.stage == 1) {
        // reconstruction status and every request's counts are on the host
        const bool bad = (int32_t)(pin[0] & 0xffffffff) != 0;
        for (size_t q2 = 0; q2 < G.reqs.size(); q2++) {
          Req &r = s->reqs[G.reqs[q2]];
          const int64_t *cn = pin + 4 + 4 * q2;
          r.nv = cn[0]; r.nt = cn[1]; r.npv = cn[2]; r.nac = cn[3];
          r.phase = 1;
          if (bad) finish(s, r, CHR_E_CORRUPT);
        }
        G.stage = 2;
      } else {
        for (int64_t id : G.reqs)
          if (s->reqs[id].phase == 2) finish(s, s->reqs[id], CHR_OK);
      }
    }
    if (!group_finished(s, G)) launch_emits(s, j);
    if (!G.inflight && group_finished(s, G)) close_group(s, j);
  }
  // Memory deadlock: every busy group waits for pool memory and none has
  // device work that will free some.  Preempt the newest group; a lone group
  // whose next request could never fit fails that request.
  int waiting = 0, active = 0, newest = -1;
  for (int j = 0; j < s->cfg.slots; j++) {
    const Group &G = s->slot[j];
    if (!G.busy) continue;
    if (G.inflight) active++;
    else {
      waiting++;
      if (newest < 0 || G.seq > s->slot[newest].seq) newest = j;
    }
  }
  if (waiting && !active) {
    if (waiting > 1) {
      preempt(s, newest);
    } else {
      // A lone group: let its first waiting request keep only the group's
      // reconstruction and its own counting state (the group's other waiting
      // requests go back to the queue); if even that cannot fit, or nothing
      // else holds memory and the free space is too fragmented, it fails.
      Group &G = s->slot[newest];
      int64_t first = -1;
      for (int64_t id : G.reqs)
        if (s->reqs[id].phase == 1) { first = id; break; }
      if (first >= 0) {
        Req &r = s->reqs[first];
        const size_t need = list_bytes(r) + mesh_bytes(r);
        const size_t held = G.recon.n + r.cstate.n;
        bool others = false;
        for (int64_t id : G.reqs)
          if (id != first && s->reqs[id].phase == 1) others = true;
        if (held + need > s->pool.bytes) {
          finish(s, r, CHR_E_NOMEM);
        } else if (others) {
          std::vector<int64_t> back;
          for (int64_t id : G.reqs) {
            Req &o = s->reqs[id];
            if (id == first || o.phase != 1) continue;
            free_block(s, o.cstate);
            o.phase = 0;
            o.state = QUEUED;
            o.group_size = 0;
            back.push_back(id);
          }
          s->queue.insert(s->queue.begin(), back.begin(), back.end());
          std::sort(s->queue.begin(), s->queue.end());
          std::vector<int64_t> keep;
          for (int64_t id : G.reqs)
            if (s->reqs[id].state != QUEUED) keep.push_back(id);
          G.reqs.swap(keep);
        } else if (s->pool.used == held) {
          finish(s, r, CHR_E_NOMEM);
        }
        launch_emits(s, newest);
        if (!G.inflight && group_finished(s, G)) close_group(s, newest);
      }
    }
  }
  // Admission only while no group waits for memory (back-pressure).
  bool any_waiting = false;
  for (int j = 0; j < s->cfg.slots; j++)
    if (s->slot[j].busy && !s->slot[j].inflight) any_waiting = true;
  if (!any_waiting)
    for (int j = 0; j < s->cfg.slots; j++)
      if (!s->slot[j].busy && !admit(s, j)) break;
  if (n_done) *n_done = (int)(s->st.done + s->st.failed - done0);
  return api_check_launch("chr_server_step");
}

int chr_server_poll(const chr_server *s, int64_t id, chr_request_result *out) {
  if (!s || !out || id < 0 || id >= (int64_t)s->reqs.size() || s->reqs[id].state == RELEASED)
    return api_fail(CHR_E_INVAL, "unknown request");
  const Req &r = s->reqs[id];
  std::memset(out, 0, sizeof(*out));
  out->status = r.status;
  out->level = r.level;
  out->dataset = r.dataset;
  out->stream_index = r.sidx;
  out->isovalue = r.k;
  out->group_size = r.group_size;
  out->error_bound = stream_bound(s->streams[r.sidx].info);
  out->t_submit_ms = r.t_submit;
  out->t_admit_ms = r.t_admit;
  out->t_done_ms = r.t_done;
  if (r.state == DONE) {
    out->n_vertices = r.nv;
    out->n_triangles = r.nt;
    const uint8_t *m = pool_ptr(s, r.mesh.off);
    out->d_vertices = reinterpret_cast<const float *>(m);
    out->d_triangles = reinterpret_cast<const int32_t *>(m + align_up(12 * (size_t)r.nv));
  }
  return CHR_OK;
}

int chr_server_release(chr_server *s, int64_t id) {
  if (!s || id < 0 || id >= (int64_t)s->reqs.size()) return api_fail(CHR_E_INVAL, "unknown request");
  Req &r = s->reqs[id];
  if (r.state == QUEUED || r.state == RUNNING) return api_fail(CHR_E_INVAL, "request not finished");
  if (r.state == RELEASED) return api_fail(CHR_E_INVAL, "request already released");
  free_block(s, r.mesh);
  r.state = RELEASED;
  return CHR_OK;
}

int chr_server_cancel(chr_server *s, int64_t id) {
  if (!s || id < 0 || id >= (int64_t)s->reqs.size()) return api_fail(CHR_E_INVAL, "unknown request");
  Req &r = s->reqs[id];
  if (r.state == QUEUED) {
    r.state = CANCELLED;
    r.status = CHR_E_CANCELLED;
    r.t_done = now_ms(s);
    s->st.failed++;
  } else if (r.state == RUNNING) {
    r.cancelled = true;
  } else {
    return api_fail(CHR_E_INVAL, "request already finished");
  }
  return CHR_OK;
}

int chr_server_stats_get(const chr_server *s, chr_server_stats *out) {
  if (!s || !out) return api_fail(CHR_E_INVAL, "NULL argument");
  *out = s->st;
  out->queued = 0;
  for (int64_t id : s->queue)
    if (s->reqs[id].state == QUEUED) out->queued++;
  out->in_flight = 0;
  for (int j = 0; j < s->cfg.slots; j++)
    if (s->slot[j].busy) out->in_flight += (int64_t)s->slot[j].reqs.size();
  out->pool_used = s->pool.used;
  out->pool_peak = s->pool.peak;
  return CHR_OK;
}

double chr_server_now_ms(const chr_server *s) { return s ? now_ms(s) : 0.0; }

int chr_server_destroy(chr_server *s) {
  if (!s) return CHR_OK;
  for (hipStream_t h : s->hs)
    if (h) hipStreamSynchronize(h);
  for (hipStream_t h : s->hs)
    if (h) hipStreamDestroy(h);
  for (hipEvent_t e : s->ev)
    if (e) hipEventDestroy(e);
  if (s->h_pinned) hipHostFree(s->h_pinned);
  delete s;
  return CHR_OK;
}

}  // extern "C"
