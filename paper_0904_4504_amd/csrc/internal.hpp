// Host-side internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lattice.hpp"
#include "lbm.h"
#include "solver.hpp"

namespace lbm {

// ds: some solve of the launch has a diffuse-scattering wall.
hipError_t launch_step(int Q, bool f64, bool bgk, bool ds, int cpt, bool outm,
                       const SolveDesc* descs, const WorkItem* work, int nwork,
                       const KernelLattice& lat, hipStream_t stream, KernelEvents ev = {});
// ds: some solve of the launch has a diffuse-scattering wall.  streaming:
// the launch's state exceeds what stays in the last-level cache between
// steps (its new coefficients then go out with nontemporal stores).
hipError_t launch_coef(int Q, bool f64, int k, bool ds, bool streaming, const SolveDesc* descs,
                       const WorkItem* work, int nwork, const KernelLattice& lat,
                       hipStream_t stream, KernelEvents ev = {});
hipError_t launch_finalize(bool f64, const SolveDesc* descs, const int32_t* solves, int nsolves,
                           int mode, hipStream_t stream);

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

inline int hip_rc(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

// Velocity set of a lattice id, host copies.
struct HostLattice {
  int Q = 0, R = 0;
  std::vector<int> vx, vy, orbit, opp;
  LatticeWeights lw{};
};

// Where every region lives inside the one device allocation.
struct Layout {
  int64_t pitch = 0, qs = 0, ys = 0, buf_elems = 0;
  int32_t ntiles = 0, cells_per_tile = kBlock, cpt = 1;
  int32_t nlinks = 0, nfcells = 0, nwcols = 0, nwlinks = 0, nlweights = 0, ncweights = 0;
  uint64_t off_links = 0, off_fcells = 0, off_wcols = 0, off_wlinks = 0;
  uint64_t off_lweights = 0, off_cweights = 0;
  // coefficient representation (mom): six coefficient planes, updated in
  // tiles of kCoefTileW columns x coef_tile_rows(coef_k) rows
  bool mom = false;
  bool loadable = true;  // has the population buffer a populations load needs
  int32_t coef_k = 0, tiles_x = 0, mntiles = 0;
  int64_t mpitch = 0, mks = 0;  // coefficient buffers: row and plane strides (elements)
  uint64_t mbuf_bytes = 0, off_mwork = 0, off_mbuf[2] = {0, 0};
  int32_t nwork = 0, mnwork = 0;  // population-kernel and coefficient-kernel work items
  int64_t hist_cap = 0;
  uint64_t off_desc = 0, off_state = 0, off_work = 0, off_solves = 0, off_drive = 0,
           off_hist = 0, off_buf[2] = {0, 0};
  uint64_t buf_bytes = 0, total = 0;
};

// Append the tiles of one solve to a launch work list in XCD-aware order
// (rows of `span` tiles dealt to the 8 XCDs in turn).
void order_tiles(std::vector<WorkItem>* out, int32_t solve, int32_t ntiles, int32_t span);
// The same tiles with each XCD taking one contiguous band of tile rows (the
// halo rows shared by vertically adjacent tiles stay in that XCD's L2);
// the same length as order_tiles.
void order_tiles_banded(std::vector<WorkItem>* out, int32_t solve, int32_t ntiles,
                        int32_t span);
// Coefficient-kernel tiles of a solve with a wall link (mask over its tiles).
std::vector<char> coef_wall_tiles(const lbm_params* p, const Layout& lay, int R);
// The tiles of one coefficient solve: its wall tiles to `front` (they are the
// slowest of a launch, so they start first), the rest to `rest` in the order
// of order_tiles_banded (banded) or order_tiles with the wall tiles made
// no-ops (keeping the XCD structure).
void order_coef_tiles(std::vector<WorkItem>* front, std::vector<WorkItem>* rest, int32_t solve,
                      const std::vector<char>& wall, int32_t ntiles, int32_t span, bool banded);
// Coefficient launches whose two state buffers together take at most this
// many bytes stay in the 256 MB last-level cache between steps: their tiles
// go in bands (reuse of the halo rows within an XCD's L2) and their stores
// are plain, so the next step reads the state from the cache.  Larger ones
// stream from HBM: the row-interleaved order (adjacent rows in flight on all
// XCDs at once) and nontemporal stores.
constexpr uint64_t kCachedStateBytes = (uint64_t)192 << 20;
// front, padded with no-ops to a multiple of 8 items, then rest.
void join_front(std::vector<WorkItem>* front, const std::vector<WorkItem>& rest);

}  // namespace lbm

struct lbm_solver;
// One step of a single solver (population, population-to-coefficient or
// coefficient kernel, then the finalize); defined in api.cpp.
int step_one(lbm_solver* s);
// Steps of a single solver captured into one graph.
constexpr int kGraphSteps = 32;

struct lbm_solver {
  // solver state; host fields mirror the device counters after a sync
  lbm_params p{};
  lbm::HostLattice lat;
  lbm::Layout lay;
  lbm::KernelLattice klat{};
  hipStream_t stream = nullptr;
  char* base = nullptr;       // device allocation (owned or caller's)
  void* bufs[2] = {nullptr, nullptr};  // population buffers; bufs[steps & 1] is current
  bool owned = false;
  int device = 0;
  int64_t steps = 0;          // steps enqueued
  bool pop_pending = false;   // coefficient solver whose current state is populations
  lbm::WorkItem* d_mwork = nullptr;   // coefficient kernel: tiles in XCD-aware order
  lbm::SolveDesc desc{};      // host copy (device pointers)
  lbm::SolveDesc* d_desc = nullptr;
  lbm::WorkItem* d_work = nullptr;
  int32_t* d_solves = nullptr;
  bool sticky_unstable = false;
  int64_t hist_from = 0;      // first step whose force is in the ring
  // graph of kGraphSteps steps (captured on first use; the launches read the
  // step index from the device, so one graph serves every later chunk)
  hipGraphExec_t graph = nullptr;
  bool graphs_ok = true;
  // device memory is the library's static scratch array of `device`
  // (lbm_create_static), released by lbm_destroy
  bool in_scratch = false;
};

namespace lbm {
// Create a solver in caller-owned device memory (dev_buf, bytes) or, with
// dev_buf null, in memory the library allocates.  graphs: lbm_step may
// capture and replay HIP graphs (off: every step launches directly).
int create_solver(const lbm_params* p, void* stream, void* dev_buf, uint64_t bytes, bool graphs,
                  lbm_solver** out);
// Mark the static scratch array of `device` free again (lbm_destroy of a
// solver created by lbm_create_static).
void release_scratch(int device);
}  // namespace lbm

