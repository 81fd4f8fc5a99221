// Batched execution: many solvers (uneven lattices, same velocity set,
// storage and collision) advanced by one fused stream-collide launch per
// step over the tiles of every member, plus one finalize launch that reduces
// each member's wall force.  Members join and leave between steps
// (continuous batching); a member stops when it reaches its max_steps.
// Steady-state chunks are replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace lbm;

struct lbm_batch {
  hipStream_t stream = nullptr;
  std::vector<lbm_solver*> members;
  int Q = 0;
  uint32_t storage = 0, collision = 0;
  int cpt = 1;
  bool have_pop = false;  // some member keeps populations (sets cpt)
  int coef_k = 0;
  bool have_mom = false;  // some member keeps coefficients (sets coef_k)
  // current launch set (members that still have steps to run)
  std::vector<lbm_solver*> active;
  bool dirty = true;
  // work items in four consecutive groups, one launch each: population
  // kernel (bounce-back wall, diffuse wall), coefficient kernel (the same);
  // every member runs the kernel instantiation it runs alone
  int ngroup[4] = {0, 0, 0, 0};
  // coefficient groups whose state streams from HBM (nontemporal stores)
  bool streaming[4] = {false, false, false, false};
  SolveDesc* d_descs = nullptr;
  WorkItem* d_work = nullptr;   // population-kernel items, then coefficient-kernel items
  int32_t* d_solves = nullptr;
  size_t cap_descs = 0, cap_work = 0, cap_solves = 0;
  // graph of `graph_steps` steps for the current launch set
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  int graph_chunk = 32;
  bool graphs_enabled = true;
  // per-launch timing of the fused step kernel
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double kernel_ms = 0;
  int64_t launches = 0;
};

namespace {

void drop_graph(lbm_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_steps = 0;
}

template <class T>
int grow(T** ptr, size_t* cap, size_t need) {
  if (need <= *cap) return LBM_OK;
  size_t n = std::max(need, *cap * 2);
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  if (hipMalloc(reinterpret_cast<void**>(ptr), n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return LBM_ENOMEM;
  }
  *cap = n;
  return LBM_OK;
}

// Rebuild the device launch set from the members that have steps left.
// Rebuild the device launch set from the given members.
int refresh(lbm_batch* b, const std::vector<lbm_solver*>& act) {
  if (!b->dirty && act == b->active) return LBM_OK;
  drop_graph(b);
  b->active = act;
  b->dirty = false;
  std::vector<SolveDesc> descs;
  // coefficient groups: every member's wall tiles first (they are the slowest
  // tiles of the launch), then the rest
  std::vector<WorkItem> group[4], front[4], work;
  std::vector<int32_t> solves;
  uint64_t state[4] = {0, 0, 0, 0};  // coefficient state bytes per group
  for (size_t i = 0; i < act.size(); ++i) {
    const Layout& lay = act[i]->lay;
    if (lay.mom) state[2 + (act[i]->p.wall != LBM_WALL_BB)] += 2 * lay.mbuf_bytes;
  }
  for (size_t i = 0; i < act.size(); ++i) {
    descs.push_back(act[i]->desc);
    solves.push_back((int32_t)i);
    const Layout& lay = act[i]->lay;
    const int k = (lay.mom ? 2 : 0) + (act[i]->p.wall != LBM_WALL_BB);
    if (lay.mom) {
      order_coef_tiles(&front[k], &group[k], (int32_t)i,
                       coef_wall_tiles(&act[i]->p, lay, act[i]->lat.R), lay.mntiles, lay.tiles_x,
                       state[k] <= kCachedStateBytes);
    } else {
      order_tiles(&group[k], (int32_t)i, lay.ntiles,
                  (act[i]->p.nx + lay.cells_per_tile - 1) / lay.cells_per_tile);
    }
  }
  for (int k = 0; k < 4; ++k) {
    if (!front[k].empty()) {
      join_front(&front[k], group[k]);
      group[k].swap(front[k]);
    }
    b->ngroup[k] = (int)group[k].size();
    b->streaming[k] = state[k] > kCachedStateBytes;
    work.insert(work.end(), group[k].begin(), group[k].end());
  }
  if (act.empty()) return LBM_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EHIP;
  int rc;
  if ((rc = grow(&b->d_descs, &b->cap_descs, descs.size()))) return rc;
  if ((rc = grow(&b->d_work, &b->cap_work, work.size()))) return rc;
  if ((rc = grow(&b->d_solves, &b->cap_solves, solves.size()))) return rc;
  if (hipMemcpy(b->d_descs, descs.data(), sizeof(SolveDesc) * descs.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_work, work.data(), sizeof(WorkItem) * work.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_solves, solves.data(), sizeof(int32_t) * solves.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return LBM_EHIP;
  return LBM_OK;
}

hipEvent_t next_event(lbm_batch* b) {
  if (b->ev_used == b->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    b->ev_pool.push_back(e);
  }
  return b->ev_pool[b->ev_used++];
}

// Sum the durations of the recorded step-kernel launches (waits).
int collect_timing(lbm_batch* b) {
  if (b->ev_used == 0) return LBM_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EHIP;
  for (size_t i = 0; i + 1 < b->ev_used; i += 2) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, b->ev_pool[i], b->ev_pool[i + 1]) != hipSuccess) return LBM_EHIP;
    b->kernel_ms += ms;
    ++b->launches;
  }
  b->ev_used = 0;
  return LBM_OK;
}

int launch_one(lbm_batch* b) {
  const bool f64 = b->storage == LBM_STORE_F64, bgk = b->collision == LBM_COLL_BGK;
  const KernelLattice& lat = b->active[0]->klat;
  int nlaunch = 0;
  for (int k = 0; k < 4; ++k) nlaunch += b->ngroup[k] > 0;
  // ev: the launch records its own start and end (it is the only step
  // kernel launch of the launch set)
  auto step = [&](KernelEvents ev) {
    const KernelEvents own = nlaunch == 1 ? ev : KernelEvents{};
    const WorkItem* work = b->d_work;
    for (int k = 0; k < 4; ++k) {
      const int n = b->ngroup[k];
      if (n == 0) continue;
      const bool ds = k & 1;
      const hipError_t e =
          k < 2 ? launch_step(b->Q, f64, bgk, ds, b->cpt, false, b->d_descs, work, n, lat,
                              b->stream, own)
                : launch_coef(b->Q, f64, b->coef_k, ds, b->streaming[k], b->d_descs, work, n,
                              lat, b->stream, own);
      if (e != hipSuccess) return e;
      work += n;
    }
    return hipSuccess;
  };
  if (b->timing) {
    if (b->ev_used + 2 > 4096) {
      int rc = collect_timing(b);
      if (rc) return rc;
    }
    hipEvent_t e0 = next_event(b), e1 = next_event(b);
    if (!e0 || !e1) return LBM_EHIP;
    if (nlaunch > 1) {
      // several launches: events around them
      if (hipEventRecord(e0, b->stream) != hipSuccess) return LBM_EHIP;
      if (step(KernelEvents{}) != hipSuccess) return LBM_EHIP;
      if (hipEventRecord(e1, b->stream) != hipSuccess) return LBM_EHIP;
    } else if (step(KernelEvents{e0, e1}) != hipSuccess) {
      return LBM_EHIP;
    }
  } else if (step(KernelEvents{}) != hipSuccess) {
    return LBM_EHIP;
  }
  if (launch_finalize(f64, b->d_descs, b->d_solves, (int)b->active.size(), 2, b->stream) !=
      hipSuccess)
    return LBM_EHIP;
  return LBM_OK;
}

// Capture graph_chunk steps of the current launch set into a graph.
bool capture(lbm_batch* b) {
  if (b->stream == nullptr) return false;  // the null stream cannot be captured
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = true;
  const bool timing = b->timing;
  b->timing = false;
  for (int k = 0; k < b->graph_chunk && ok; ++k) ok = launch_one(b) == LBM_OK;
  b->timing = timing;
  if (hipStreamEndCapture(b->stream, &g) != hipSuccess || !ok) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  hipGraphExec_t ex = nullptr;
  const bool inst = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!inst) {
    (void)hipGetLastError();
    return false;
  }
  b->graph = ex;
  b->graph_steps = b->graph_chunk;
  return true;
}

}  // namespace

extern "C" {

int lbm_batch_create(void* hip_stream, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->stream = static_cast<hipStream_t>(hip_stream);
  *out = b;
  return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, lbm_solver* s) {
  if (!b || !s) return LBM_EINVAL;
  if (s->stream != b->stream) return LBM_EINVAL;
  if (std::find(b->members.begin(), b->members.end(), s) != b->members.end()) return LBM_EINVAL;
  if (b->members.empty()) {
    b->Q = (int)s->p.lattice;
    b->storage = s->p.storage;
    b->collision = s->p.collision;
  } else if ((int)s->p.lattice != b->Q || s->p.storage != b->storage ||
             s->p.collision != b->collision) {
    return LBM_EINVAL;
  }
  // members kept as populations share one population-kernel launch, members
  // kept as coefficients one coefficient-kernel launch
  if (!s->lay.mom) {
    if (b->have_pop && s->lay.cpt != b->cpt) return LBM_EINVAL;
    b->have_pop = true;
    b->cpt = s->lay.cpt;
  } else {
    if (b->have_mom && s->lay.coef_k != b->coef_k) return LBM_EINVAL;
    b->have_mom = true;
    b->coef_k = s->lay.coef_k;
  }
  b->members.push_back(s);
  b->dirty = true;
  return LBM_OK;
}

int lbm_batch_remove(lbm_batch* b, lbm_solver* s) {
  if (!b || !s) return LBM_EINVAL;
  auto it = std::find(b->members.begin(), b->members.end(), s);
  if (it == b->members.end()) return LBM_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EHIP;
  b->members.erase(it);
  b->dirty = true;
  if (b->members.empty()) {
    b->Q = 0;
    b->have_pop = false;
    b->have_mom = false;
  }
  return LBM_OK;
}

int lbm_batch_size(const lbm_batch* b, int* members, int* active) {
  if (!b) return LBM_EINVAL;
  if (members) *members = (int)b->members.size();
  if (active) {
    int n = 0;
    for (lbm_solver* s : b->members) n += s->steps < s->p.max_steps;
    *active = n;
  }
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  // steps each member still takes in this call
  std::vector<int64_t> left(b->members.size());
  for (size_t i = 0; i < b->members.size(); ++i) {
    lbm_solver* s = b->members[i];
    left[i] = std::min(nsteps, s->p.max_steps - s->steps);
    // a coefficient member whose state was just loaded as populations takes
    // that step alone (population kernel writing coefficients)
    if (s->pop_pending && left[i] > 0) {
      int rc = step_one(s);
      if (rc) return rc;
      --left[i];
    }
  }
  for (;;) {
    std::vector<lbm_solver*> act;
    int64_t chunk = 0;
    for (size_t i = 0; i < b->members.size(); ++i)
      if (left[i] > 0) {
        act.push_back(b->members[i]);
        chunk = chunk ? std::min(chunk, left[i]) : left[i];
      }
    if (act.empty()) break;
    int rc = refresh(b, act);
    if (rc) return rc;
    int64_t k = 0;
    if (b->graphs_enabled && !b->timing && chunk >= b->graph_chunk) {
      if (!b->graph && !capture(b)) b->graphs_enabled = false;
      for (; b->graph && k + b->graph_steps <= chunk; k += b->graph_steps)
        if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return LBM_EHIP;
    }
    for (; k < chunk; ++k)
      if ((rc = launch_one(b))) return rc;
    for (size_t i = 0; i < b->members.size(); ++i)
      if (left[i] > 0) {
        b->members[i]->steps += chunk;
        left[i] -= chunk;
      }
  }
  return LBM_OK;
}

int lbm_batch_synchronize(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EHIP;
  int worst = LBM_OK;
  for (lbm_solver* s : b->members) {
    int rc = lbm_synchronize(s);
    if (rc && !worst) worst = rc;
  }
  return worst;
}

int lbm_batch_set_graphs(lbm_batch* b, int steps_per_graph) {
  if (!b || steps_per_graph < 0) return LBM_EINVAL;
  drop_graph(b);
  b->graphs_enabled = steps_per_graph > 0;
  if (steps_per_graph > 0) b->graph_chunk = steps_per_graph;
  return LBM_OK;
}

int lbm_batch_timing(lbm_batch* b, int enable) {
  if (!b) return LBM_EINVAL;
  int rc = collect_timing(b);
  b->timing = enable != 0;
  b->kernel_ms = 0;
  b->launches = 0;
  return rc;
}

int lbm_batch_kernel_time(lbm_batch* b, double* ms, int64_t* launches) {
  if (!b) return LBM_EINVAL;
  int rc = collect_timing(b);
  if (ms) *ms = b->kernel_ms;
  if (launches) *launches = b->launches;
  return rc;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  int rc = hipStreamSynchronize(b->stream) == hipSuccess ? LBM_OK : LBM_EHIP;
  drop_graph(b);
  for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_solves) (void)hipFree(b->d_solves);
  delete b;
  return rc;
}

}  // extern "C"
