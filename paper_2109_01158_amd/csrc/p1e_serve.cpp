// p1e_serve.cpp -- host side of the multi-request engine: the continuous-batching server
// (p1e_server_*) and the single-request minimizer (p1e_minimize).
//
// A server owns one caller-provided device pool. Its head holds the engine tables (slot
// descriptors, per-slot scalars, tile tables); the rest is handed out to requests first-fit.
// Requests are built on host worker threads (mesh setup), admitted in arrival order when a
// slot and enough pool bytes are free, advanced together one line-search trial per engine step
// (a fixed launch sequence, optionally replayed from a captured hipGraph), and retired when
// their iteration budget is spent. Admission and retirement only rewrite the tables between
// steps, so the captured graph stays valid.
//
// The minimization follows the paper's use of J and grad J in a first-order method (Section 7,
// where the paper uses a trust-region method): here L-BFGS with memory m, Armijo
// backtracking by halving and a first step of largest nodal update 0.1 h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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

#include "p1e_admission.h"
#include "p1e_internal.h"

using namespace p1e;

namespace {

uint64_t aup(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int class_of(const p1e_mesh *m) {
  if (m->kind == P1E_NEOHOOKE) return m->dim == 3 ? CLS_NH3 : CLS_NH2;
  return m->dim == 3 ? CLS_PLAP3 : CLS_PLAP2;
}

// mesh size for the first step: the edge of the smallest element's reference cell,
// (dim! |T|_min)^(1/dim)
double mesh_h(const p1e_mesh *m) {
  const double f = m->dim == 3 ? 6.0 : 2.0;
  return m->min_vol > 0.0 ? std::pow(f * m->min_vol, 1.0 / m->dim) : 1.0;
}

// bytes of the L-BFGS state of one slot after its mesh arrays
uint64_t state_bytes(const p1e_mesh *m, int history) {
  const uint64_t n = (uint64_t)std::max<int64_t>(m->nfd, 1);
  const uint64_t ntv = (n + kVecTile - 1) / kVecTile;
  return aup(5 * n * 8) + aup(2ull * history * n * 8) + aup(ntv * kNPart * 16) + aup(8ull * kNSyy);
}

// capacities of the tile tables for a workspace of pool_bytes: every element tile but a
// mesh's last holds at least 12 KiB of slot data (1024 elements or 1024 nodes), every
// halo-row tile (kBlock rows) at least 32 KiB (gradient, load and L-BFGS vectors per row);
// plus one partial tile per slot
struct TableCaps {
  int64_t slots, tile, halo, vec;
};
TableCaps table_caps(int max_slots, uint64_t pool_bytes) {
  TableCaps c;
  c.slots = max_slots;
  c.tile = (int64_t)(pool_bytes / 12288) + 2 * max_slots;
  c.halo = (int64_t)(pool_bytes / 32768) + 2 * max_slots;
  c.vec = (int64_t)(pool_bytes / (kVecTile * 64)) + 2 * max_slots;
  return c;
}
int64_t halo_tiles(const p1e_mesh *m) { return (m->nhalo + kBlock - 1) / kBlock; }
// exact capacities for one slot holding mesh m
TableCaps table_caps_for(const p1e_mesh *m) {
  TableCaps c;
  c.slots = 1;
  c.tile = m->ntiles + 1;
  c.halo = halo_tiles(m) + 1;
  c.vec = (std::max<int64_t>(m->nfd, 1) + kVecTile - 1) / kVecTile + 1;
  return c;
}
uint64_t table_bytes(const TableCaps &c) {
  return aup(sizeof(SlotDev) * c.slots) + aup(8ull * kNSc * c.slots) + aup(4ull * kNSt * c.slots) +
         aup(8ull * c.tile) + aup(8ull * c.halo) + aup(8ull * c.vec) + aup(4ull * kNumCounts);
}

// ---------------------------------------------------------------------------- engine
// Tables and slot bookkeeping shared by the server and the single-request minimizer.
struct Engine {
  EngineDev E{};
  TableCaps caps{};
  hipStream_t stream = nullptr;
  std::vector<SlotDev> slots_h;
  std::vector<int> cls_h;         // class of each slot (-1 = free)
  std::vector<double> sc_h;       // host copies read back after a step (pinned)
  std::vector<int32_t> st_h;
  double *sc_pin = nullptr;
  int32_t *st_pin = nullptr;
  bool tables_dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;

  int init(char *base, uint64_t bytes, const TableCaps &tc, int history, int prec, hipStream_t s,
           bool graph_on) {
    caps = tc;
    const int max_slots = (int)tc.slots;
    if (table_bytes(caps) > bytes) return fail(P1E_ENOMEM, "workspace too small for the engine tables");
    stream = s;
    use_graph = graph_on;
    uint64_t off = 0;
    auto take = [&](uint64_t n) {
      char *p = base + off;
      off += aup(n);
      return p;
    };
    E.slots = (SlotDev *)take(sizeof(SlotDev) * max_slots);
    E.sc = (double *)take(8ull * kNSc * max_slots);
    E.st = (int32_t *)take(4ull * kNSt * max_slots);
    E.map[TK_TILE] = (int2 *)take(8ull * caps.tile);
    E.map[TK_HALO] = (int2 *)take(8ull * caps.halo);
    E.vmap = (int2 *)take(8ull * caps.vec);
    E.counts = (int32_t *)take(4ull * kNumCounts);
    E.max_slots = max_slots;
    E.history = history;
    E.prec = prec;
    slots_h.assign(max_slots, SlotDev{});
    cls_h.assign(max_slots, -1);
    sc_h.assign((size_t)kNSc * max_slots, 0.0);
    st_h.assign((size_t)kNSt * max_slots, 0);
    if (hipHostMalloc((void **)&sc_pin, 8ull * kNSc * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&st_pin, 4ull * kNSt * max_slots) != hipSuccess)
      return fail(P1E_EHIP, "pinned host buffers");
    std::memset(sc_pin, 0, 8ull * kNSc * max_slots);
    std::memset(st_pin, 0, 4ull * kNSt * max_slots);
    if (hipMemcpyAsync(E.sc, sc_pin, 8ull * kNSc * max_slots, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(E.st, st_pin, 4ull * kNSt * max_slots, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(P1E_EHIP, "engine table upload");
    tables_dirty = true;
    return P1E_OK;
  }

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    if (sc_pin) (void)hipHostFree(sc_pin);
    if (st_pin) (void)hipHostFree(st_pin);
    sc_pin = nullptr;
    st_pin = nullptr;
  }

  // occupy slot k with a bound mesh (m->dev) and its state arrays at `state`
  int attach(int k, p1e_mesh *m, char *state, const double *vhat0_dev, const double *vhat0_host,
             int max_iters) {
    const int64_t n = m->nfd;
    const uint64_t n1 = (uint64_t)std::max<int64_t>(n, 1);
    SlotDev S{};
    S.M = m->dev;
    S.ntile_h = (int)halo_tiles(m);
    S.ntile_v = (int)((n + kVecTile - 1) / kVecTile);
    S.C1 = m->C1;
    S.D1 = m->D1;
    S.p = m->p;
    S.ortho = m->ortho;
    S.dirichlet_bv = m->dirichlet_bv;
    uint64_t off = 0;
    auto take = [&](uint64_t b) {
      char *p = state + off;
      off += aup(b);
      return p;
    };
    char *vec5 = take(5 * n1 * 8);
    S.v = (double *)vec5;
    S.g = S.v + n1;
    S.d = S.g + n1;
    S.vt = S.d + n1;
    S.gt = S.vt + n1;
    char *hist = take(2ull * E.history * n1 * 8);
    S.S = (double *)hist;
    S.Y = S.S + (uint64_t)E.history * n1;
    S.vpart = (double2 *)take((uint64_t)S.ntile_v * kNPart * 16);
    S.syy = (double *)take(8ull * kNSyy);
    slots_h[k] = S;
    cls_h[k] = class_of(m);
    // state rows
    double *sc = sc_pin + (size_t)k * kNSc;
    int32_t *st = st_pin + (size_t)k * kNSt;
    std::memset(sc, 0, 8ull * kNSc);
    std::memset(st, 0, 4ull * kNSt);
    sc[SC_H] = mesh_h(m);
    st[ST_MODE] = MODE_INIT;
    st[ST_MAXIT] = max_iters;
    st[ST_HEAD] = E.history - 1;
    st[ST_CLASS] = cls_h[k];
    bool ok = hipMemcpyAsync(E.sc + (size_t)k * kNSc, sc, 8ull * kNSc, hipMemcpyHostToDevice, stream) == hipSuccess &&
              hipMemcpyAsync(E.st + (size_t)k * kNSt, st, 4ull * kNSt, hipMemcpyHostToDevice, stream) == hipSuccess;
    if (n > 0) {
      hipMemcpyKind kind = vhat0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
      const void *src = vhat0_dev ? (const void *)vhat0_dev : (const void *)vhat0_host;
      ok = ok && hipMemcpyAsync(S.v, src, 8ull * n, kind, stream) == hipSuccess &&
           hipMemcpyAsync(S.vt, src, 8ull * n, kind, stream) == hipSuccess;
    }
    if (!ok) return fail(P1E_EHIP, "slot upload failed");
    tables_dirty = true;
    return P1E_OK;
  }

  int detach(int k) {
    cls_h[k] = -1;
    slots_h[k] = SlotDev{};
    int32_t *st = st_pin + (size_t)k * kNSt;
    std::memset(st, 0, 4ull * kNSt);
    st[ST_MODE] = MODE_FREE;
    if (hipMemcpyAsync(E.st + (size_t)k * kNSt, st, 4ull * kNSt, hipMemcpyHostToDevice, stream) != hipSuccess)
      return fail(P1E_EHIP, "slot release failed");
    tables_dirty = true;
    return P1E_OK;
  }

  // rebuild and upload the tile tables of the occupied slots
  int upload_tables() {
    if (!tables_dirty) return P1E_OK;
    std::vector<int2> maps[kNumTileKinds];
    std::vector<int2> vmap;
    std::vector<int32_t> counts(kNumCounts, 0);
    for (int kind = 0; kind < kNumTileKinds; ++kind)
      for (int c = 0; c < kNumClasses; ++c) {
        counts[2 * (kind * kNumClasses + c)] = (int32_t)maps[kind].size();
        for (int k = 0; k < E.max_slots; ++k) {
          if (cls_h[k] != c) continue;
          const SlotDev &S = slots_h[k];
          const int n = kind == TK_TILE ? S.M.ntiles : S.ntile_h;
          for (int t = 0; t < n; ++t) maps[kind].push_back(make_int2(k, t));
        }
        counts[2 * (kind * kNumClasses + c) + 1] =
            (int32_t)maps[kind].size() - counts[2 * (kind * kNumClasses + c)];
      }
    for (int k = 0; k < E.max_slots; ++k)
      if (cls_h[k] >= 0)
        for (int t = 0; t < slots_h[k].ntile_v; ++t) vmap.push_back(make_int2(k, t));
    counts[kCountVec] = (int32_t)vmap.size();
    if ((int64_t)maps[TK_TILE].size() > caps.tile || (int64_t)maps[TK_HALO].size() > caps.halo ||
        (int64_t)vmap.size() > caps.vec)
      return fail(P1E_ENOMEM, "tile tables over capacity");
    bool ok = hipMemcpyAsync(E.slots, slots_h.data(), sizeof(SlotDev) * E.max_slots,
                             hipMemcpyHostToDevice, stream) == hipSuccess;
    for (int kind = 0; kind < kNumTileKinds; ++kind)
      if (!maps[kind].empty())
        ok = ok && hipMemcpyAsync(E.map[kind], maps[kind].data(), 8ull * maps[kind].size(),
                                  hipMemcpyHostToDevice, stream) == hipSuccess;
    if (!vmap.empty())
      ok = ok && hipMemcpyAsync(E.vmap, vmap.data(), 8ull * vmap.size(), hipMemcpyHostToDevice,
                                stream) == hipSuccess;
    ok = ok && hipMemcpyAsync(E.counts, counts.data(), 4ull * kNumCounts, hipMemcpyHostToDevice,
                              stream) == hipSuccess;
    // pageable sources: make sure the copies are done before the vectors go away
    ok = ok && hipStreamSynchronize(stream) == hipSuccess;
    if (!ok) return fail(P1E_EHIP, "table upload failed");
    tables_dirty = false;
    return P1E_OK;
  }

  // one engine step, then an asynchronous copy of the slot states to pinned host memory
  int step() {
    int rc = upload_tables();
    if (rc) return rc;
    if (use_graph) {
      if (!exec) {
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
          return fail(P1E_EHIP, "graph capture begin");
        rc = batch_step(E, stream);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(stream, &g) != hipSuccess || rc)
          return rc ? rc : fail(P1E_EHIP, "graph capture end");
        graph = g;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
          return fail(P1E_EHIP, "graph instantiate");
      }
      if (hipGraphLaunch(exec, stream) != hipSuccess) return fail(P1E_EHIP, "graph launch");
    } else {
      rc = batch_step(E, stream);
      if (rc) return rc;
    }
    if (hipMemcpyAsync(st_pin, E.st, 4ull * kNSt * E.max_slots, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(sc_pin, E.sc, 8ull * kNSc * E.max_slots, hipMemcpyDeviceToHost, stream) != hipSuccess)
      return fail(P1E_EHIP, "state readback");
    return P1E_OK;
  }

  int wait() {
    if (hipStreamSynchronize(stream) != hipSuccess)
      return fail(P1E_EHIP, std::string("engine step failed: ") + hipGetErrorString(hipGetLastError()));
    return P1E_OK;
  }
};

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------- server
struct p1e_server {
  p1e_server_opts opts{};
  Engine eng;
  char *data = nullptr;  // request area of the pool
  uint64_t data_bytes = 0;
  Admission adm;  // slots and first-fit blocks of the request area
  double t0 = 0.0;

  struct Req {
    int64_t id = 0;
    double t_arrival = 0.0;  // server clock; not built or admitted before
    p1e_mesh_desc desc{};
    std::vector<int32_t> conn;
    std::vector<double> coords, dvals, load, vhat0;
    std::vector<uint8_t> dmask;
    p1e_mesh *mesh = nullptr;
    int setup_rc = P1E_OK;
    std::string setup_err;
    p1e_request_info info{};
    uint64_t off = 0, bytes = 0;
    int slot = -1;
    std::vector<double> vhat;
  };
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req *> to_build;
  std::map<int64_t, Req *> ready;     // built, waiting for admission (arrival order)
  std::vector<Req *> in_slot;         // per slot
  std::map<int64_t, Req *> finished;  // waiting for poll / release
  std::deque<int64_t> unpolled;
  std::vector<std::thread> workers;
  bool stopping = false;
  int64_t next_id = 1;
  int64_t building = 0;
  bool inflight = false;

  ~p1e_server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = true;
    }
    cv.notify_all();
    for (auto &t : workers) t.join();
    if (inflight) (void)eng.wait();
    for (auto *r : to_build) delete r;
    for (auto &kv : ready) {
      p1e_mesh_destroy(kv.second->mesh);
      delete kv.second;
    }
    for (auto *r : in_slot)
      if (r) {
        p1e_mesh_destroy(r->mesh);
        delete r;
      }
    for (auto &kv : finished) delete kv.second;
    eng.release();
  }

  void worker() {
    for (;;) {
      Req *r;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stopping) return;
          if (!to_build.empty()) {
            const double wait = to_build.front()->t_arrival - (now_s() - t0);
            if (wait <= 0.0) break;
            cv.wait_for(lk, std::chrono::duration<double>(std::min(wait, 0.01)));
          } else {
            cv.wait(lk);
          }
        }
        r = to_build.front();
        to_build.pop_front();
      }
      r->setup_rc = p1e_mesh_create(&r->desc, &r->mesh);
      if (r->setup_rc != P1E_OK) r->setup_err = p1e_last_error();
      r->conn.clear();
      r->coords.clear();
      r->dvals.clear();
      r->load.clear();
      r->dmask.clear();
      if (r->mesh) {
        r->bytes = aup(p1e_workspace_bytes(r->mesh, opts.prec)) + state_bytes(r->mesh, opts.history);
        if (r->vhat0.empty()) {  // default start: prescribed values and v = x (Neo-Hookean) or 0
          r->vhat0.assign(r->mesh->nfd, 0.0);
          if (r->mesh->kind == P1E_NEOHOOKE) {
            // the free components of node i keep x in wref (internal order)
            for (int64_t i = 0; i < r->mesh->nn; ++i) {
              int info = r->mesh->ninfo[i];
              int mask = info & 7;
              int64_t fb = info >> 3;
              for (int j = 0; j < r->mesh->d; ++j)
                if (mask >> j & 1) r->vhat0[fb++] = r->mesh->wref[i * r->mesh->d + j];
            }
          }
        }
      }
      std::lock_guard<std::mutex> lk(mu);
      ready[r->id] = r;
      --building;
    }
  }

};

extern "C" {

uint64_t p1e_server_table_bytes(int32_t max_slots, uint64_t pool_bytes) {
  if (max_slots < 1) return 0;
  return table_bytes(table_caps(max_slots, pool_bytes));
}

int p1e_server_create(const p1e_server_opts *o, p1e_server **out) {
  if (!o || !out) return fail(P1E_EINVAL, "null argument");
  *out = nullptr;
  if (o->max_slots < 1 || o->max_slots > 4096) return fail(P1E_EINVAL, "max_slots out of range");
  if (o->history < 1 || o->history > kMaxHistory) return fail(P1E_EINVAL, "history out of range");
  if (o->max_iters < 0) return fail(P1E_EINVAL, "max_iters < 0");
  if (o->prec != P1E_FP64 && o->prec != P1E_MIXED) return fail(P1E_EINVAL, "prec");
  if (!o->pool || (uintptr_t)o->pool % kAlign) return fail(P1E_EINVAL, "pool must be 256-byte aligned");
  std::unique_ptr<p1e_server> S(new p1e_server());
  S->opts = *o;
  const uint64_t tb = table_bytes(table_caps(o->max_slots, o->pool_bytes));
  if (tb >= o->pool_bytes) return fail(P1E_ENOMEM, "pool too small for the engine tables");
  if (o->use_graph && !o->stream) return fail(P1E_EINVAL, "graph capture needs a non-default stream");
  int rc = S->eng.init((char *)o->pool, tb, table_caps(o->max_slots, o->pool_bytes), o->history,
                       o->prec, (hipStream_t)o->stream, o->use_graph != 0);
  if (rc) return rc;
  S->data = (char *)o->pool + tb;
  S->data_bytes = o->pool_bytes - tb;
  S->adm.reset(o->max_slots, S->data_bytes);
  S->in_slot.assign(o->max_slots, nullptr);
  S->t0 = now_s();
  const int nt = std::max(1, (int)o->setup_threads);
  for (int i = 0; i < nt; ++i) S->workers.emplace_back([p = S.get()] { p->worker(); });
  *out = S.release();
  return P1E_OK;
}

void p1e_server_destroy(p1e_server *s) { delete s; }

double p1e_server_clock(const p1e_server *s) { return s ? now_s() - s->t0 : 0.0; }

int p1e_server_submit_at(p1e_server *s, const p1e_mesh_desc *d, const double *vhat0,
                         int64_t n0, double t_arrival, int64_t *id) {
  if (!s || !d || !id) return fail(P1E_EINVAL, "null argument");
  if (d->dim != 2 && d->dim != 3) return fail(P1E_EINVAL, "dim must be 2 or 3");
  if (d->kind != P1E_PLAPLACE && d->kind != P1E_PLAPLACE_ORTHO && d->kind != P1E_NEOHOOKE)
    return fail(P1E_EINVAL, "the server covers the p-Laplacian and Neo-Hookean kinds");
  if (d->nn < 1 || d->ne < 0 || !d->coords || (d->ne > 0 && !d->conn))
    return fail(P1E_EINVAL, "bad mesh description");
  const int k = d->dim + 1;
  const int nc = d->ncomp;
  if (nc < 1 || nc > 3) return fail(P1E_EINVAL, "ncomp");
  auto *r = new p1e_server::Req();
  r->desc = *d;
  r->conn.assign(d->conn, d->conn + (size_t)d->ne * k);
  r->coords.assign(d->coords, d->coords + (size_t)d->nn * d->dim);
  if (d->dirichlet) r->dmask.assign(d->dirichlet, d->dirichlet + (size_t)d->nn * nc);
  if (d->dirichlet_values) r->dvals.assign(d->dirichlet_values, d->dirichlet_values + (size_t)d->nn * nc);
  if (d->load) r->load.assign(d->load, d->load + (size_t)d->nn * nc);
  if (vhat0 && n0 > 0) r->vhat0.assign(vhat0, vhat0 + n0);
  r->desc.conn = r->conn.empty() ? nullptr : r->conn.data();
  r->desc.coords = r->coords.data();
  r->desc.dirichlet = r->dmask.empty() ? nullptr : r->dmask.data();
  r->desc.dirichlet_values = r->dvals.empty() ? nullptr : r->dvals.data();
  r->desc.load = r->load.empty() ? nullptr : r->load.data();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->info.id = r->id;
    r->t_arrival = std::max(t_arrival, now_s() - s->t0);
    r->info.t_submit = r->t_arrival;
    // building order = arrival order
    auto pos = std::upper_bound(s->to_build.begin(), s->to_build.end(), r,
                                [](const p1e_server::Req *a, const p1e_server::Req *b) {
                                  return a->t_arrival < b->t_arrival;
                                });
    s->to_build.insert(pos, r);
    ++s->building;  // submitted and not yet built (includes requests still to arrive)
    *id = r->id;
  }
  s->cv.notify_one();
  return P1E_OK;
}

int p1e_server_submit(p1e_server *s, const p1e_mesh_desc *d, const double *vhat0, int64_t n0,
                      int64_t *id) {
  return p1e_server_submit_at(s, d, vhat0, n0, 0.0, id);
}

int p1e_server_step(p1e_server *s, int32_t *n_active, int32_t *n_waiting) {
  if (!s) return fail(P1E_EINVAL, "null server");
  Engine &E = s->eng;
  int rc;
  // 1. results of the previous step
  if (s->inflight) {
    rc = E.wait();
    s->inflight = false;
    if (rc) return rc;
    for (int k = 0; k < E.E.max_slots; ++k) {
      p1e_server::Req *r = s->in_slot[k];
      if (!r) continue;
      const int32_t *st = E.st_pin + (size_t)k * kNSt;
      if (st[ST_MODE] != MODE_DONE) continue;
      const double *sc = E.sc_pin + (size_t)k * kNSc;
      r->info.status = st[ST_STATUS];
      r->info.iterations = st[ST_ITER];
      r->info.evaluations = st[ST_EVALS];
      r->info.J = sc[SC_J];
      r->info.J_grad = sc[SC_JG];
      r->vhat.resize(r->mesh->nfd);
      if (r->mesh->nfd > 0 &&
          hipMemcpy(r->vhat.data(), E.slots_h[k].v, 8ull * r->mesh->nfd, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(P1E_EHIP, "result readback");
      r->info.t_done = now_s() - s->t0;
      rc = E.detach(k);
      if (rc) return rc;
      s->adm.retire(k, r->off, r->bytes);
      p1e_mesh_destroy(r->mesh);
      r->mesh = nullptr;
      s->in_slot[k] = nullptr;
      std::lock_guard<std::mutex> lk(s->mu);
      s->finished[r->id] = r;
      s->unpolled.push_back(r->id);
    }
  }
  // 2. admission in arrival order while a slot and pool bytes are free
  for (;;) {
    p1e_server::Req *r = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->ready.empty()) break;
      r = s->ready.begin()->second;
    }
    if (r->setup_rc != P1E_OK) {  // failed setup: finish at once with its status
      std::lock_guard<std::mutex> lk(s->mu);
      s->ready.erase(r->id);
      r->info.status = r->setup_rc;
      r->info.t_admit = r->info.t_done = now_s() - s->t0;
      s->finished[r->id] = r;
      s->unpolled.push_back(r->id);
      continue;
    }
    int k = -1;
    uint64_t off = 0;
    const Admit a = s->adm.try_admit(r->id, r->bytes, k, off);
    if (a == Admit::kNever) {  // larger than the whole request area
      std::lock_guard<std::mutex> lk(s->mu);
      s->ready.erase(r->id);
      r->info.status = P1E_ENOMEM;
      r->info.t_admit = r->info.t_done = now_s() - s->t0;
      p1e_mesh_destroy(r->mesh);
      r->mesh = nullptr;
      s->finished[r->id] = r;
      s->unpolled.push_back(r->id);
      continue;
    }
    if (a == Admit::kWait) break;  // no slot or no block yet: wait for a retirement
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->ready.erase(r->id);
    }
    r->off = off;
    r->slot = k;
    const uint64_t wb = aup(p1e_workspace_bytes(r->mesh, s->opts.prec));
    rc = p1e_mesh_bind(r->mesh, s->data + off, wb, s->opts.prec, s->opts.stream);
    if (rc) return rc;
    rc = E.attach(k, r->mesh, s->data + off + wb, nullptr, r->vhat0.data(), s->opts.max_iters);
    if (rc) return rc;
    r->vhat0.clear();
    r->vhat0.shrink_to_fit();
    r->info.t_admit = now_s() - s->t0;
    r->info.n_free_dofs = (int32_t)r->mesh->nfd;
    r->info.device_bytes = r->bytes;
    s->in_slot[k] = r;
  }
  // 3. one step for every active slot
  int active = 0;
  for (auto *r : s->in_slot) active += r != nullptr;
  if (active) {
    rc = E.step();
    if (rc) return rc;
    s->inflight = true;
  }
  if (n_active) *n_active = active;
  if (n_waiting) {
    std::lock_guard<std::mutex> lk(s->mu);
    *n_waiting = (int32_t)(s->ready.size() + s->building);
  }
  return P1E_OK;
}

int p1e_server_run(p1e_server *s, int64_t max_steps, double max_seconds, int32_t *n_active,
                   int32_t *n_waiting) {
  if (!s) return fail(P1E_EINVAL, "null server");
  const double t_end = now_s() + (max_seconds > 0.0 ? max_seconds : 1e300);
  int32_t a = 0, w = 0;
  for (int64_t k = 0; max_steps <= 0 || k < max_steps; ++k) {
    int rc = p1e_server_step(s, &a, &w);
    if (rc) return rc;
    if (a == 0 && w == 0 && !s->inflight) break;
    if (now_s() > t_end) break;
    if (a == 0) std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  if (n_active) *n_active = a;
  if (n_waiting) *n_waiting = w;
  return P1E_OK;
}

int p1e_server_poll(p1e_server *s, p1e_request_info *out, int32_t cap, int32_t *n) {
  if (!s || !n || (cap > 0 && !out)) return fail(P1E_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t c = 0;
  while (c < cap && !s->unpolled.empty()) {
    out[c++] = s->finished[s->unpolled.front()]->info;
    s->unpolled.pop_front();
  }
  *n = c;
  return P1E_OK;
}

int p1e_server_result_vhat(p1e_server *s, int64_t id, double *dst, int64_t n) {
  if (!s || (!dst && n > 0)) return fail(P1E_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->finished.find(id);
  if (it == s->finished.end()) return fail(P1E_EINVAL, "unknown or unfinished request");
  if ((int64_t)it->second->vhat.size() != n) return fail(P1E_EINVAL, "length mismatch");
  if (n) std::memcpy(dst, it->second->vhat.data(), 8ull * n);
  return P1E_OK;
}

int p1e_server_release(p1e_server *s, int64_t id) {
  if (!s) return fail(P1E_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->finished.find(id);
  if (it == s->finished.end()) return fail(P1E_EINVAL, "unknown or unfinished request");
  delete it->second;
  s->finished.erase(it);
  return P1E_OK;
}

// ---------------------------------------------------------------------------- minimize
uint64_t p1e_minimize_workspace_bytes(const p1e_mesh *m, const p1e_lbfgs_opts *o) {
  if (!m || !o || o->history < 1 || o->history > kMaxHistory) return 0;
  return table_bytes(table_caps_for(m)) + state_bytes(m, o->history);
}

int p1e_minimize(p1e_mesh *m, double *vhat, const p1e_lbfgs_opts *o, void *ws, uint64_t ws_bytes,
                 p1e_min_report *rep, void *stream) {
  if (!m || !o || !ws || !rep || (!vhat && m->nfd > 0)) return fail(P1E_EINVAL, "null argument");
  if (o->history < 1 || o->history > kMaxHistory || o->max_iters < 0)
    return fail(P1E_EINVAL, "bad L-BFGS options");
  if (o->prec != P1E_FP64 && o->prec != P1E_MIXED) return fail(P1E_EINVAL, "prec");
  if (m->kind != P1E_PLAPLACE && m->kind != P1E_NEOHOOKE)
    return fail(P1E_EINVAL, "the minimizer covers the p-Laplacian and Neo-Hookean kinds");
  if (!(m->bound_modes & o->prec)) return fail(P1E_ESTATE, "mesh not bound for the requested precision");
  if ((uintptr_t)ws % kAlign) return fail(P1E_EINVAL, "workspace must be 256-byte aligned");
  const uint64_t need = p1e_minimize_workspace_bytes(m, o);
  if (ws_bytes < need) return fail(P1E_ENOMEM, "workspace too small");
  const uint64_t tb = table_bytes(table_caps_for(m));
  Engine E;
  hipStream_t s = (hipStream_t)stream;
  int rc = E.init((char *)ws, tb, table_caps_for(m), o->history, o->prec, s, false);
  if (rc) {
    E.release();
    return rc;
  }
  m->forces_prec = 0;  // the engine overwrites the mesh's scratch arrays
  rc = E.attach(0, m, (char *)ws + tb, vhat, nullptr, o->max_iters);
  int64_t steps = 0;
  const int64_t max_steps = (int64_t)(o->max_iters + 1) * (kMaxLineTrials + 1) + 1;
  while (rc == P1E_OK) {
    rc = E.step();
    if (rc) break;
    rc = E.wait();
    if (rc || E.st_pin[ST_MODE] == MODE_DONE || ++steps > max_steps) break;
  }
  if (rc == P1E_OK) {
    rep->status = E.st_pin[ST_STATUS];
    rep->iterations = E.st_pin[ST_ITER];
    rep->evaluations = E.st_pin[ST_EVALS];
    rep->J = E.sc_pin[SC_J];
    rep->J_grad = E.sc_pin[SC_JG];
    if (m->nfd > 0 &&
        (hipMemcpyAsync(vhat, E.slots_h[0].v, 8ull * m->nfd, hipMemcpyDeviceToDevice, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
      rc = fail(P1E_EHIP, "result copy failed");
    if (rep->status == SLOT_BAD_START) rc = fail(P1E_EDOMAIN, "no admissible start (bad elements)");
  }
  E.release();
  return rc;
}

}  // extern "C"
