// Host-side internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lattice.hpp"
#include "lbm.h"
#include "solver.hpp"

namespace lbm {

hipError_t launch_step(int Q, bool f64, bool bgk, int cpt, const SolveDesc* descs,
                       const WorkItem* work, int nwork, const KernelLattice& lat,
                       hipStream_t stream);
hipError_t launch_finalize(const SolveDesc* descs, const int32_t* solves, int nsolves,
                           hipStream_t stream);

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
  int32_t ntiles = 0, nslots = 0, cells_per_tile = kBlock, cpt = 1;
  int64_t hist_cap = 0;
  uint64_t off_desc = 0, off_state = 0, off_work = 0, off_solves = 0, off_slot = 0,
           off_part = 0, off_drive = 0, off_hist = 0, off_buf[2] = {0, 0};
  uint64_t buf_bytes = 0, total = 0;
};

}  // namespace lbm

struct lbm_solver {
  // solver state; host fields mirror the device counters after a sync
  lbm_params p{};
  lbm::HostLattice lat;
  lbm::Layout lay;
  lbm::KernelLattice klat{};
  hipStream_t stream = nullptr;
  char* base = nullptr;       // device allocation (owned or caller's)
  bool owned = false;
  int device = 0;
  int64_t steps = 0;          // steps enqueued
  lbm::SolveDesc desc{};      // host copy (device pointers)
  lbm::SolveDesc* d_desc = nullptr;
  lbm::WorkItem* d_work = nullptr;
  int32_t* d_solves = nullptr;
  bool sticky_unstable = false;
  int64_t hist_from = 0;      // first step whose force is in the ring
};

