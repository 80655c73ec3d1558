// stb_server.hip -- continuous-batching request server on device-resident
// meshes: matvec (16 right-hand sides) and potential requests.
//
// Slots: each slot is a worker thread with a context of its own (stream,
// pair-pipeline workspace, events), so the work of requests on different
// slots overlaps on the device.  A request is admitted as soon as a slot is
// free and its device footprint fits the HBM budget beside the requests in
// flight (continuous batching: requests that arrive while others run join
// as slots and memory free up, instead of waiting for a batch boundary).
// The kernels are deterministic and a request touches no state shared with
// other requests except the read-only meshes and matrices, so its result is
// the same alone and in a mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "stb_internal.h"
#include "stb_pairs.h"

using namespace stb;

namespace {

using Clock = std::chrono::steady_clock;

struct Ticket {
  stb_request req;
  Clock::time_point t_submit;
  double latency_s = 0.0;
  stb_status status = STB_OK;
  bool done = false;
  std::string err;
};

struct ServedMesh {
  stb_mesh* mesh;
  stb_mat* mat;   // may be NULL (potential requests only)
};

}  // namespace

struct stb_server {
  stb_ctx* ctx = nullptr;
  // in_use: the requests in flight plus every slot's pipeline workspace
  // (held between requests; slot_ws[k] of it belongs to slot k)
  int64_t budget = 0, in_use = 0;
  std::vector<stb_ctx*> slots;
  std::vector<int64_t> slot_ws;
  std::vector<std::thread> workers;
  // a deque: registering a mesh never moves the ones already served
  std::deque<ServedMesh> meshes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int64_t completed = 0;
};

namespace {

// Device bytes a request needs while it runs, beyond the slot's own
// workspace: its inputs and outputs, and for a potential the cull's
// candidate arrays (one int64 row pointer per point, column + row + value
// per candidate, counted exactly by a cull pass).
int64_t matvec_bytes(const stb_mat* M) { return M->n * 16 * (8 + 8 + 4); }

int64_t potential_bytes(int64_t nt, int64_t np, int64_t nnz) {
  return nt * 8 + np * (32 + 8 + 64 + 8) + nnz * (4 + 4 + 8);
}

stb_status run_request(stb_ctx* c, const ServedMesh& sm, const stb_request& r, std::string* err) {
  hipStream_t st = c->stream;
  stb_status s = STB_OK;
  if (r.kind == STB_REQ_MATVEC16) {
    const int64_t n = sm.mat->n;
    double *w = nullptr, *y = nullptr;
    if (dalloc(&w, (size_t)n * 16) != hipSuccess || dalloc(&y, (size_t)n * 16) != hipSuccess) {
      dfree(w); dfree(y);
      return stb_fail(c, STB_E_NO_MEMORY, "matvec buffers");
    }
    hipError_t e = hipMemcpyAsync(w, r.w, sizeof(double) * n * 16, hipMemcpyHostToDevice, st);
    s = e == hipSuccess ? stb_apply16_dev(c, sm.mat, w, y, st) : stb_fail(c, STB_E_DEVICE, "copy in");
    if (s == STB_OK) {
      e = hipMemcpyAsync(r.out, y, sizeof(double) * n * 16, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) s = stb_fail(c, STB_E_DEVICE, "copy out: %s", hipGetErrorString(e));
    }
    dfree(w);
    dfree(y);
  } else {
    const int64_t nt = sm.mesh->nt;
    double *w = nullptr, *pts = nullptr, *u = nullptr;
    if (dalloc(&w, (size_t)nt) != hipSuccess || dalloc(&pts, (size_t)r.np * 4) != hipSuccess ||
        dalloc(&u, (size_t)r.np) != hipSuccess) {
      dfree(w); dfree(pts); dfree(u);
      return stb_fail(c, STB_E_NO_MEMORY, "potential buffers");
    }
    hipError_t e = hipMemcpyAsync(w, r.w, sizeof(double) * nt, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pts, r.pts, sizeof(double) * 4 * r.np, hipMemcpyHostToDevice, st);
    stb_quad_params p = stb_default_params();
    s = e == hipSuccess ? stb_potential_core(c, sm.mesh, p, w, r.np, pts, u)
                        : stb_fail(c, STB_E_DEVICE, "copy in");
    if (s == STB_OK) {
      e = hipMemcpyAsync(r.out, u, sizeof(double) * r.np, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) s = stb_fail(c, STB_E_DEVICE, "copy out: %s", hipGetErrorString(e));
    }
    dfree(w);
    dfree(pts);
    dfree(u);
  }
  if (s) *err = c->err;
  return s;
}

// Exact footprint of a request (a potential needs its cull count): its own
// buffers (*bytes) and the size slot context c's pipeline workspace will
// have after it (*ws).
stb_status footprint(stb_ctx* c, const ServedMesh& sm, const stb_request& r, int64_t* bytes,
                     int64_t* ws) {
  *ws = stb_pairs_ws_held(c);
  if (r.kind == STB_REQ_MATVEC16) {
    *bytes = matvec_bytes(sm.mat);
    return STB_OK;
  }
  // the points' lit search, as the request will run it, for its count
  double* pts = nullptr;
  if (dalloc(&pts, (size_t)r.np * 4) != hipSuccess) return stb_fail(c, STB_E_NO_MEMORY, "footprint buffers");
  stb_status s = STB_OK;
  int64_t nnz = 0;
  hipError_t e = hipMemcpyAsync(pts, r.pts, sizeof(double) * 4 * r.np, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    int64_t* rp = nullptr;
    int32_t *cols = nullptr, *rowof = nullptr;
    stb_quad_params p = stb_default_params();
    s = stb_cull_points(c, sm.mesh, p, r.np, pts, &rp, &cols, &rowof, &nnz);
    dfree(rp); dfree(cols); dfree(rowof);
  } else {
    s = stb_fail(c, STB_E_DEVICE, "copy in");
  }
  dfree(pts);
  *bytes = potential_bytes(sm.mesh->nt, r.np, nnz);
  *ws = stb_pairs_ws_need(c, nnz, 1);
  return s;
}

void worker(stb_server* S, int slot) {
  stb_ctx* c = S->slots[(size_t)slot];
  (void)hipSetDevice(c->device);
  for (;;) {
    uint64_t id = 0;
    stb_request r;
    ServedMesh sm{};
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
      if (S->queue.empty()) return;   // stopping and drained
      id = S->queue.front();
      S->queue.pop_front();
      r = S->tickets[id].req;
      sm = S->meshes[(size_t)r.mesh];   // a copy, taken under the lock
    }
    std::string err;
    int64_t bytes = 0, ws = 0;
    stb_status s = footprint(c, sm, r, &bytes, &ws);
    int64_t grow = 0;
    if (s == STB_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      grow = std::max<int64_t>(0, ws - S->slot_ws[(size_t)slot]);
      // the other slots' workspaces stay held while this request runs
      const int64_t others = [&] {
        int64_t o = 0;
        for (size_t k = 0; k < S->slot_ws.size(); ++k)
          if ((int)k != slot) o += S->slot_ws[k];
        return o;
      }();
      if (bytes + ws + others > S->budget)
        s = stb_fail(c, STB_E_NO_MEMORY, "request needs %lld bytes (+%lld of workspace), budget %lld",
                     (long long)bytes, (long long)ws, (long long)S->budget);
    }
    if (s == STB_OK) {
      // admission by HBM footprint: the request's buffers and the growth of
      // this slot's workspace beside everything already in use
      {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_mem.wait(lk, [&] { return S->in_use + bytes + grow <= S->budget; });
        S->in_use += bytes + grow;
        S->slot_ws[(size_t)slot] += grow;
      }
      s = run_request(c, sm, r, &err);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= bytes;
        // the workspace the slot really holds now (it may have been sized down
        // to fit the device)
        const int64_t held = stb_pairs_ws_held(c);
        S->in_use += held - S->slot_ws[(size_t)slot];
        S->slot_ws[(size_t)slot] = held;
      }
      S->cv_mem.notify_all();
    } else {
      err = c->err;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      Ticket& t = S->tickets[id];
      t.status = s;
      t.err = err;
      t.latency_s = std::chrono::duration<double>(Clock::now() - t.t_submit).count();
      t.done = true;
      ++S->completed;
    }
    S->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

stb_status stb_server_create(stb_ctx* ctx, int64_t hbm_budget_bytes, int32_t nslots,
                             stb_server** out) {
  if (!ctx || !out || nslots < 1 || nslots > 16 || hbm_budget_bytes < 0)
    return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments (1 <= nslots <= 16, budget >= 0)");
  *out = nullptr;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(ctx, hipMemGetInfo(&fr, &tot));
    hbm_budget_bytes = (int64_t)(0.5 * (double)fr);
  }
  stb_server* S = new stb_server();
  S->ctx = ctx;
  S->budget = hbm_budget_bytes;
  for (int k = 0; k < nslots; ++k) {
    stb_ctx* c = nullptr;
    stb_status s = stb_ctx_create(ctx->device, &c);
    if (s) {
      for (auto* x : S->slots) stb_ctx_destroy(x);
      delete S;
      return stb_fail(ctx, s, "slot context: %s", stb_last_error(nullptr));
    }
    for (int q = 0; q < 8; ++q) {   // the parent's launch shapes
      c->tune_block[q] = ctx->tune_block[q];
      c->tune_per_cu[q] = ctx->tune_per_cu[q];
    }
    c->tuned = ctx->tuned;
    S->slots.push_back(c);
    S->slot_ws.push_back(0);
  }
  for (int k = 0; k < nslots; ++k) S->workers.emplace_back(worker, S, k);
  *out = S;
  return STB_OK;
}

stb_status stb_server_add_mesh(stb_server* S, const stb_mesh* mesh, const stb_mat* mat, int32_t* id) {
  if (!S || !mesh || !id) return stb_fail(S ? S->ctx : nullptr, STB_E_INVALID_ARG, "NULL argument");
  if (mesh->ctx != S->ctx || (mat && mat->ctx != S->ctx))
    return stb_fail(S->ctx, STB_E_INVALID_ARG, "mesh or matrix of another context");
  if (mat && mat->n != mesh->nt) return stb_fail(S->ctx, STB_E_INVALID_ARG, "matrix size != mesh size");
  stb_mat* M = const_cast<stb_mat*>(mat);
  if (M && !M->d_bptr) {
    // the matrix-core copy is built once here, not by concurrent requests
    stb_status s = stb_build_blocked(S->ctx, M, S->ctx->stream);
    if (s) return s;
    HIPCHK(S->ctx, hipStreamSynchronize(S->ctx->stream));
  }
  {
    // the lit-search tree for the requests' parameters, built once here
    const stb_quad_params p = stb_default_params();
    if (p.lit_search == STB_LIT_TREE) {
      stb_status s = stb_ensure_tree(S->ctx, const_cast<stb_mesh*>(mesh), p.n_min);
      if (s) return s;
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->meshes.push_back({const_cast<stb_mesh*>(mesh), M});
  *id = (int32_t)(S->meshes.size() - 1);
  return STB_OK;
}

stb_status stb_server_submit(stb_server* S, const stb_request* req, uint64_t* ticket) {
  if (!S || !req || !ticket) return stb_fail(S ? S->ctx : nullptr, STB_E_INVALID_ARG, "NULL argument");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (req->mesh < 0 || (size_t)req->mesh >= S->meshes.size())
      return stb_fail(nullptr, STB_E_NOT_FOUND, "unknown mesh id %d", req->mesh);
    const ServedMesh& sm = S->meshes[(size_t)req->mesh];
    if (req->kind == STB_REQ_MATVEC16) {
      if (!sm.mat) return stb_fail(nullptr, STB_E_INVALID_ARG, "mesh %d has no matrix", req->mesh);
      if (!req->w || !req->out) return stb_fail(nullptr, STB_E_INVALID_ARG, "matvec needs w and out");
    } else if (req->kind == STB_REQ_POTENTIAL) {
      if (req->np < 1 || !req->w || !req->pts || !req->out)
        return stb_fail(nullptr, STB_E_INVALID_ARG, "potential needs np >= 1, w, pts, out");
    } else {
      return stb_fail(nullptr, STB_E_INVALID_ARG, "unknown request kind %d", req->kind);
    }
    if (S->stopping) return stb_fail(nullptr, STB_E_BUSY, "server is shutting down");
    uint64_t id = S->next_ticket++;
    Ticket& t = S->tickets[id];
    t.req = *req;
    t.t_submit = Clock::now();
    S->queue.push_back(id);
    *ticket = id;
  }
  S->cv_work.notify_one();
  return STB_OK;
}

stb_status stb_server_wait(stb_server* S, uint64_t ticket, double* latency_s) {
  if (!S) return stb_fail(nullptr, STB_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return stb_fail(nullptr, STB_E_NOT_FOUND, "unknown ticket %llu",
                                              (unsigned long long)ticket);
  S->cv_done.wait(lk, [&] { return it->second.done; });
  stb_status s = it->second.status;
  if (latency_s) *latency_s = it->second.latency_s;
  if (s) stb_fail(nullptr, s, "%s", it->second.err.c_str());
  S->tickets.erase(it);
  return s;
}

void stb_server_destroy(stb_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto* c : S->slots) stb_ctx_destroy(c);
  delete S;
}

}  // extern "C"
