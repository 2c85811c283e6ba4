// Batched Heun step: thousands of independent 1D/2D/3D problems, each with
// its own grid, time step and CFL reduction, packed into one buffer.
//
// The plan cuts every problem into work items (1D: rows of 63 cells; 2D:
// 63-cell row segments walking a range of rows; 3D: x-y tiles walking a
// range of z planes).  Each stage is one persistent launch sized to the
// resident capacity of the machine, and the plan deals the items to its
// workgroups by the longest-processing-time rule: most expensive item first,
// each to the workgroup with the least work so far.  Workgroup b runs the
// contiguous run [start[b], start[b+1]) of the item list (no shared counter,
// no atomics to hand out work).  The item body is the single-grid
// tile body (stage_tile.hpp).  In stage 2 each item stores the CFL signal
// max of its cells into its own slot; a small kernel then reduces the slots
// of each problem into the problem's next dt.  Nothing needs clearing
// between launches, so the step can be captured in a graph.  1D and 2D
// problems share one launch (one wave per item); 3D problems (heavier
// tiles, more registers) get their own.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <queue>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hard.h"
#include "api_internal.hpp"
#include "hydro_device.hpp"
#include "launch.hpp"
#include "stage_tile.hpp"

namespace hard {

struct BatchProblem {
  long long offset;  // element offset of the problem's state in the packed buffer
  int n[3];
  int ndim;
  int bc[3][2];
  double dx[3];
  double inv_dx[3];
  int dx_pow2;
  int tiles_x, tiles_y, nchunk, ntiles;  // work items of this problem
  int walk;                              // walk positions per work item (2D rows, 3D planes)
  int slot0;                             // first CFL slot of the problem (one per item)
};

struct WorkItem {
  int prob;
  int tile;
};

struct BatchArgs {
  const void* src;
  const void* un;
  void* dst;
  const BatchProblem* probs;
  const WorkItem* items;
  int nitems;
  const int* start;  // stage kernels: workgroup b runs items [start[b], start[b+1])
  double* dt;        // per-problem dt (read)
  double* slot;      // per-item CFL signal max (written when the item computes it)
  Control* ctl;      // status bits
  double gamma;
  int fuse_cfl;      // stage 2: store the CFL signal max of the new state
};

// 1D and 2D problems: one wave per work item.  A 1D item is a row of 63
// cells (64 faces, one per lane); a 2D item is a row segment of 63 cells
// walking along y over `walk` rows.
constexpr int BT12 = 64;
constexpr int ROW = BT12 - 1;
// 3D problems: 256-thread workgroups, x-y tiles walking along z.
constexpr int BT3 = 256;
constexpr int kTiles3D[3][2] = {{16, 16}, {32, 8}, {8, 32}};

// Item-level finish: status bits to the control block, the item's CFL
// signal max to its slot.
template <int NTHR>
__device__ __forceinline__ void tile_finish(unsigned flags, double smax, bool do_cfl,
                                            const BatchArgs& a, int slot) {
  constexpr int NW = NTHR / 64;
  flags = wave_or(flags);
  if (do_cfl) smax = wave_max(smax);
  if constexpr (NW == 1) {
    if (threadIdx.x == 0) {
      if (flags) atomicOr(&a.ctl->flags, flags);
      if (do_cfl) a.slot[slot] = smax;
    }
  } else {
    __shared__ double red_s[NW];
    __shared__ unsigned red_f[NW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red_f[w] = flags;
      red_s[w] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned f = 0;
      double m = 0.0;
      for (int i = 0; i < NW; ++i) {
        f |= red_f[i];
        m = fmax(m, red_s[i]);
      }
      if (f) atomicOr(&a.ctl->flags, f);
      if (do_cfl) a.slot[slot] = m;
    }
    __syncthreads();  // red_* are reused by the next item
  }
}

__device__ __forceinline__ TileArgs tile_args(const BatchArgs& a, const BatchProblem& P, int wsize) {
  TileArgs t;
  t.src = static_cast<const char*>(a.src) + P.offset * wsize;
  t.un = static_cast<const char*>(a.un) + P.offset * wsize;
  t.dst = static_cast<char*>(a.dst) + P.offset * wsize;
  for (int k = 0; k < 3; ++k) {
    t.n[k] = P.n[k];
    t.bc[k][0] = P.bc[k][0];
    t.bc[k][1] = P.bc[k][1];
    t.dx[k] = P.dx[k];
    t.inv_dx[k] = P.inv_dx[k];
  }
  t.dx_pow2 = P.dx_pow2;
  t.gamma = a.gamma;
  t.exchange = 0;  // batched problems carry no radiation field
  t.kappa = 0.0;
  t.mu = 1.0;
  return t;
}

// Work item -> tile origin and walk range.  1D: x row; 2D: x row segment and
// a range of rows; 3D: x-y tile and a range of planes.
__device__ __forceinline__ void item_geometry(const BatchProblem& P, int tile, int tx_cells,
                                              int ty_cells, TileArgs& t) {
  const int txi = tile % P.tiles_x;
  const int rest = tile / P.tiles_x;
  const int tyi = rest % P.tiles_y;
  const int chunk = rest / P.tiles_y;
  t.x0 = txi * tx_cells;
  t.y0 = P.ndim == 3 ? tyi * ty_cells : 0;
  const int nwalk = P.ndim == 3 ? P.n[2] : (P.ndim == 2 ? P.n[1] : 1);
  t.w0 = P.ndim >= 2 ? chunk * P.walk : 0;
  t.w1 = P.ndim >= 2 ? min(t.w0 + P.walk, nwalk) : 1;
}

template <typename R, int STAGE>
__global__ __launch_bounds__(BT12) void batched_stage_12(BatchArgs a) {
  constexpr int L1 = TileShape<1, R, ROW, 1>::lds_elems;
  constexpr int L2 = TileShape<2, R, ROW, 1>::lds_elems;
  __shared__ R lds[L1 > L2 ? L1 : L2];
  const bool do_cfl = STAGE == 2 && a.fuse_cfl;
  const int i1 = a.start[blockIdx.x + 1];
  for (int it = a.start[blockIdx.x]; it < i1; ++it) {
    const WorkItem w = a.items[it];
    const BatchProblem P = a.probs[w.prob];
    TileArgs t = tile_args(a, P, sizeof(R));
    t.dt = a.dt[w.prob];
    t.fuse_cfl = do_cfl;
    item_geometry(P, w.tile, ROW, 1, t);
    unsigned flags = 0;
    double smax = 0.0;
    if (P.ndim == 1)
      run_tile<1, R, STAGE, ROW, 1, BT12>(t, lds, flags, smax);
    else
      run_tile<2, R, STAGE, ROW, 1, BT12>(t, lds, flags, smax);
    tile_finish<BT12>(flags, smax, do_cfl, a, P.slot0 + w.tile);
    __syncthreads();  // the next item rewrites lds
  }
}

template <typename R, int STAGE, int TS>
__global__ __launch_bounds__(BT3) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 3 : 1, 8)))
void batched_stage_3(BatchArgs a) {
  constexpr int TX = kTiles3D[TS][0], TY = kTiles3D[TS][1];
  __shared__ R lds[TileShape<3, R, TX, TY>::lds_elems];
  const bool do_cfl = STAGE == 2 && a.fuse_cfl;
  const int i1 = a.start[blockIdx.x + 1];
  for (int it = a.start[blockIdx.x]; it < i1; ++it) {
    const WorkItem w = a.items[it];
    const BatchProblem P = a.probs[w.prob];
    TileArgs t = tile_args(a, P, sizeof(R));
    t.dt = a.dt[w.prob];
    t.fuse_cfl = do_cfl;
    item_geometry(P, w.tile, TX, TY, t);
    unsigned flags = 0;
    double smax = 0.0;
    run_tile<3, R, STAGE, TX, TY, BT3>(t, lds, flags, smax);
    tile_finish<BT3>(flags, smax, do_cfl, a, P.slot0 + w.tile);
    __syncthreads();
  }
}

// CFL signal max of the current state (standalone), item by item, into the
// items' slots.
template <typename R, int NTHR>
__global__ __launch_bounds__(NTHR) void batched_cfl(BatchArgs a, int tx3, int ty3) {
  for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
    const WorkItem w = a.items[it];
    const BatchProblem P = a.probs[w.prob];
    const R* U = reinterpret_cast<const R*>(static_cast<const char*>(a.src) + P.offset * sizeof(R));
    const long long N = (long long)P.n[0] * P.n[1] * P.n[2];
    const int txc = P.ndim == 3 ? tx3 : ROW;
    const int tyc = P.ndim == 3 ? ty3 : 1;
    TileArgs t;
    item_geometry(P, w.tile, txc, tyc, t);
    double smax = 0.0;
    unsigned flags = 0;
    const int tid = threadIdx.x;
    const int gx = t.x0 + tid % txc, gy = P.ndim == 3 ? t.y0 + tid / txc : 0;
    const int NV = P.ndim + 2;
    if (tid < txc * tyc && gx < P.n[0] && (P.ndim != 3 || gy < P.n[1])) {
      for (int ww = t.w0; ww < t.w1; ++ww) {
        long long c = P.ndim == 3 ? ((long long)ww * P.n[1] + gy) * P.n[0] + gx
                                  : (long long)ww * P.n[0] + gx;
        double Ud[5];
        R Ur[5], W[5];
        for (int v = 0; v < 5; ++v) {
          Ur[v] = v < NV ? U[v * N + c] : R(0);
          Ud[v] = (double)Ur[v];
        }
        if (P.ndim == 1) {
          to_primitive<R, 1>(Ur, W, a.gamma - 1.0);
          flags |= cell_flags<R, 3>(Ur, W[2]);
          smax = fmax(smax, cfl_signal<R, 1>(Ud, P.inv_dx, a.gamma));
        } else if (P.ndim == 2) {
          to_primitive<R, 2>(Ur, W, a.gamma - 1.0);
          flags |= cell_flags<R, 4>(Ur, W[3]);
          smax = fmax(smax, cfl_signal<R, 2>(Ud, P.inv_dx, a.gamma));
        } else {
          to_primitive<R, 3>(Ur, W, a.gamma - 1.0);
          flags |= cell_flags<R, 5>(Ur, W[4]);
          smax = fmax(smax, cfl_signal<R, 3>(Ud, P.inv_dx, a.gamma));
        }
      }
    }
    tile_finish<NTHR>(flags, smax, true, a, P.slot0 + w.tile);
  }
}

// dt of every problem from its items' slots: cfl / max(slot), one wave per
// problem (a problem's slots are contiguous; the max does not depend on the
// order it is taken in).
constexpr int DT_FINAL_THREADS = 256;
__global__ __launch_bounds__(DT_FINAL_THREADS) void batched_dt_final(int nprob,
                                                                     const BatchProblem* probs,
                                                                     const double* slot,
                                                                     double cfl, double* dt) {
  const int p = blockIdx.x * (DT_FINAL_THREADS / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= nprob) return;  // the whole wave
  const int s0 = probs[p].slot0, ns = probs[p].ntiles;
  double m = 0.0;
  for (int i = lane; i < ns; i += 64) m = fmax(m, slot[s0 + i]);
  m = wave_max(m);
  if (lane == 0) dt[p] = cfl / m;
}

// Per-problem time control of hard_run_batched: clip dt so each problem
// lands on t_end, advance its t, and turn its steps after the end into dt = 0
// (exact no-ops).  `active` counts the problems that took a real step.
__global__ void batched_time_control(int nprob, double* dt, double* t, long long* steps,
                                     double t_end, long long max_steps, unsigned* active) {
#pragma clang fp contract(off)
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  double tp = t[p];
  long long s = steps[p];
  if (!(tp < t_end * (1.0 - 1e-14)) || s >= max_steps) {
    dt[p] = 0.0;
    return;
  }
  double d = dt[p];
  if (d > t_end - tp) d = t_end - tp;
  dt[p] = d;
  t[p] = tp + d;
  steps[p] = s + 1;
  atomicAdd(active, 1u);
}

__global__ void batched_run_clear(int nprob, double* t, long long* steps, unsigned* active) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) *active = 0u;
  if (p < nprob) {
    t[p] = 0.0;
    steps[p] = 0;
  }
}

__global__ void counter_clear(unsigned* c) {
  if (threadIdx.x == 0) *c = 0u;
}

}  // namespace hard

using namespace hard;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct hard_batch_plan {
  int nprob = 0;
  int dtype = 0;
  double gamma = 0;
  int wsize = 8;
  int tile3d = 0;   // index into kTiles3D (x-y tile of 3D problems)
  int walk2d = 64;  // rows per 2D work item
  int cz = 32;      // planes per 3D work item
  std::vector<int64_t> offsets;
  long long total_elems = 0;
  int nitems12 = 0, nitems3 = 0;
  BatchProblem* d_probs = nullptr;
  WorkItem* d_items12 = nullptr;
  WorkItem* d_items3 = nullptr;
  int* d_start12 = nullptr;  // grid12 + 1 item offsets, one run per workgroup
  int* d_start3 = nullptr;
  int grid12 = 0, grid3 = 0;
  // workspace layout
  size_t ws_ctl = 0, ws_active = 0, ws_slot = 0, ws_t = 0, ws_steps = 0, ws_stage = 0,
         ws_total = 0;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tile choices from a tune cache, lines "key = value":
//   walk2d = 64          rows per 2D work item
//   tile3d_f64 = 16x16   x-y tile of 3D problems (tile3d_f32 for float)
//   cz = 32              planes per 3D work item
static void read_tune_cache(const char* path, hard_batch_plan* P) {
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  const std::string key3 = P->dtype == HARD_F64 ? "tile3d_f64" : "tile3d_f32";
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string k, eq, v;
    if (!(ss >> k >> eq >> v) || eq != "=") continue;
    if (k == key3) {
      int x = 0, y = 0;
      if (std::sscanf(v.c_str(), "%dx%d", &x, &y) == 2)
        for (int i = 0; i < 3; ++i)
          if (kTiles3D[i][0] == x && kTiles3D[i][1] == y) P->tile3d = i;
    } else if (k == "walk2d") {
      int c = std::atoi(v.c_str());
      if (c > 0 && c <= 65536) P->walk2d = c;
    } else if (k == "cz") {
      int c = std::atoi(v.c_str());
      if (c > 0 && c <= 65536) P->cz = c;
    }
  }
}

// Longest-processing-time dealing of work items to G workgroups: the items
// in decreasing cost (ties in list order), each to the workgroup with the
// least cost so far (ties: the lowest index).  Returns the items grouped by
// workgroup and the G + 1 run offsets.
struct CostedItem {
  double c;
  WorkItem w;
};
static void deal_items(std::vector<CostedItem>& v, int G, std::vector<WorkItem>& items,
                       std::vector<int>& start) {
  std::stable_sort(v.begin(), v.end(),
                   [](const CostedItem& a, const CostedItem& b) { return a.c > b.c; });
  using Load = std::pair<double, int>;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int b = 0; b < G; ++b) heap.push({0.0, b});
  std::vector<int> owner(v.size()), count(G, 0);
  for (size_t i = 0; i < v.size(); ++i) {
    const Load l = heap.top();
    heap.pop();
    owner[i] = l.second;
    ++count[l.second];
    heap.push({l.first + v[i].c, l.second});
  }
  start.assign(G + 1, 0);
  for (int b = 0; b < G; ++b) start[b + 1] = start[b] + count[b];
  std::vector<int> pos(start.begin(), start.end() - 1);
  items.resize(v.size());
  for (size_t i = 0; i < v.size(); ++i) items[pos[owner[i]]++] = v[i].w;
}

static hard_status_t batch_common(const hard_batch_plan_t* P, const void* U, const double* dt,
                                  void* work, size_t work_bytes, BatchArgs* a) {
  if (!P) return fail(HARD_ERR_INVALID_ARG, "plan is NULL");
  hard_status_t st;
  if ((st = check_ptr(U, 256, "U"))) return st;
  if ((st = check_ptr(dt, 8, "dt_dev"))) return st;
  if ((st = check_work(work, work_bytes, P->ws_total))) return st;
  char* wb = static_cast<char*>(work);
  std::memset(a, 0, sizeof *a);
  a->probs = P->d_probs;
  a->dt = const_cast<double*>(dt);
  a->slot = reinterpret_cast<double*>(wb + P->ws_slot);
  a->ctl = reinterpret_cast<Control*>(wb + P->ws_ctl);
  a->gamma = P->gamma;
  return HARD_OK;
}

static hipError_t launch_dt_final(const hard_batch_plan_t* P, const BatchArgs& a, double cfl,
                                  hipStream_t s) {
  constexpr int per_block = DT_FINAL_THREADS / 64;
  const int nb = (P->nprob + per_block - 1) / per_block;
  hipLaunchKernelGGL(batched_dt_final, dim3(nb), dim3(DT_FINAL_THREADS), 0, s, P->nprob,
                     (const BatchProblem*)P->d_probs, (const double*)a.slot, cfl, a.dt);
  return hipGetLastError();
}

template <typename R, int STAGE>
static hipError_t launch_batched_stage(const hard_batch_plan_t* P, BatchArgs a, char* wb,
                                       hipStream_t s) {
  if (P->nitems12) {
    BatchArgs b = a;
    b.items = P->d_items12;
    b.nitems = P->nitems12;
    b.start = P->d_start12;
    hipLaunchKernelGGL((batched_stage_12<R, STAGE>), dim3(P->grid12), dim3(BT12), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (P->nitems3) {
    BatchArgs b = a;
    b.items = P->d_items3;
    b.nitems = P->nitems3;
    b.start = P->d_start3;
    switch (P->tile3d) {
      case 0: hipLaunchKernelGGL((batched_stage_3<R, STAGE, 0>), dim3(P->grid3), dim3(BT3), 0, s, b); break;
      case 1: hipLaunchKernelGGL((batched_stage_3<R, STAGE, 1>), dim3(P->grid3), dim3(BT3), 0, s, b); break;
      default: hipLaunchKernelGGL((batched_stage_3<R, STAGE, 2>), dim3(P->grid3), dim3(BT3), 0, s, b); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" {

hard_status_t hard_batch_plan_create(const hard_grid_t* grids, int32_t nprob,
                                     const char* tune_cache, hard_batch_plan_t** out) {
  if (!out) return fail(HARD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grids || nprob < 1) return fail(HARD_ERR_INVALID_ARG, "need at least one grid");
  auto* P = new hard_batch_plan;
  P->nprob = nprob;
  P->dtype = grids[0].dtype;
  P->gamma = grids[0].gamma;
  P->wsize = P->dtype == HARD_F64 ? 8 : 4;
  P->tile3d = P->dtype == HARD_F64 ? 0 : 1;
  read_tune_cache(tune_cache, P);
  const int TX3 = kTiles3D[P->tile3d][0], TY3 = kTiles3D[P->tile3d][1];
  std::vector<BatchProblem> probs(nprob);
  std::vector<CostedItem> c12, c3;
  P->offsets.resize(nprob + 1);
  long long off = 0, nslot = 0;
  for (int p = 0; p < nprob; ++p) {
    Grid G;
    hard_status_t st = check_grid(&grids[p], &G);
    if (st) {
      delete P;
      return fail(st, "grid %d: %s", p, hard_last_error());
    }
    if (G.scheme != HARD_SCHEME_MUSCL_HLLC || G.rad) {
      delete P;
      return fail(HARD_ERR_UNSUPPORTED, "grid %d: the batched step is built for HARD_SCHEME_MUSCL_HLLC without radiation", p);
    }
    if (G.dtype != P->dtype || G.gamma != P->gamma) {
      delete P;
      return fail(HARD_ERR_INVALID_ARG, "grid %d: all grids must share dtype and gamma", p);
    }
    BatchProblem& B = probs[p];
    B.offset = off;
    P->offsets[p] = off;
    B.ndim = G.ndim;
    for (int d = 0; d < 3; ++d) {
      B.n[d] = G.n[d];
      B.bc[d][0] = G.bc[d][0];
      B.bc[d][1] = G.bc[d][1];
      B.dx[d] = G.dx[d];
      B.inv_dx[d] = G.inv_dx[d];
    }
    B.dx_pow2 = G.dx_pow2;
    int nwalk;  // walk positions of the problem (1 in 1D)
    if (G.ndim == 1) {
      B.tiles_x = (G.n[0] + ROW - 1) / ROW;
      B.tiles_y = 1;
      B.walk = 1;
      B.nchunk = 1;
      nwalk = 1;
    } else if (G.ndim == 2) {
      B.tiles_x = (G.n[0] + ROW - 1) / ROW;
      B.tiles_y = 1;
      B.walk = P->walk2d;
      B.nchunk = (G.n[1] + B.walk - 1) / B.walk;
      nwalk = G.n[1];
    } else {
      B.tiles_x = (G.n[0] + TX3 - 1) / TX3;
      B.tiles_y = (G.n[1] + TY3 - 1) / TY3;
      B.walk = P->cz;
      B.nchunk = (G.n[2] + B.walk - 1) / B.walk;
      nwalk = G.n[2];
    }
    B.ntiles = B.tiles_x * B.tiles_y * B.nchunk;
    B.slot0 = (int)nslot;
    nslot += B.ntiles;
    if (nslot > (1LL << 30)) {
      delete P;
      return fail(HARD_ERR_INVALID_ARG, "batch has more than 2^30 work items");
    }
    // Cost of an item in walk positions of its tile: a wave takes a row (or
    // a workgroup a plane) in about the same time however many of its lanes
    // hold cells, so the cost is the positions the item walks, plus two for
    // its set-up and prologue (four positions loaded, one face computed).
    const int per_chunk = B.tiles_x * B.tiles_y;
    for (int t = 0; t < B.ntiles; ++t) {
      const int chunk = t / per_chunk;
      const double cost = std::min(B.walk, nwalk - chunk * B.walk) + 2.0;
      (G.ndim == 3 ? c3 : c12).push_back({cost, {p, t}});
    }
    // keep every problem 256-byte aligned
    long long elems = (long long)G.nvar * G.ncell;
    long long align = 256 / P->wsize;
    off += (elems + align - 1) / align * align;
  }
  P->offsets[nprob] = off;
  P->total_elems = off;
  P->nitems12 = (int)c12.size();
  P->nitems3 = (int)c3.size();
  // persistent grids: the resident capacity of the machine for the stage-2
  // kernel (the larger register footprint), at most one workgroup per item
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 256;
  int occ12 = 0, occ3 = 0;
  if (P->dtype == HARD_F64) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ12, batched_stage_12<double, 2>, BT12, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ3, batched_stage_3<double, 2, 0>, BT3, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ12, batched_stage_12<float, 2>, BT12, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ3, batched_stage_3<float, 2, 1>, BT3, 0);
  }
  occ12 = std::max(1, std::min(occ12, 32));
  occ3 = std::max(1, std::min(occ3, 8));
  P->grid12 = std::max(1, std::min(P->nitems12, ncu * occ12));
  P->grid3 = std::max(1, std::min(P->nitems3, ncu * occ3));
  std::vector<WorkItem> i12, i3;
  std::vector<int> s12, s3;
  deal_items(c12, P->grid12, i12, s12);
  deal_items(c3, P->grid3, i3, s3);
  hipError_t e;
  if ((e = hipMalloc(&P->d_probs, sizeof(BatchProblem) * nprob)) != hipSuccess ||
      (e = hipMalloc(&P->d_items12, sizeof(WorkItem) * std::max(1, P->nitems12))) != hipSuccess ||
      (e = hipMalloc(&P->d_items3, sizeof(WorkItem) * std::max(1, P->nitems3))) != hipSuccess ||
      (e = hipMalloc(&P->d_start12, sizeof(int) * (P->grid12 + 1))) != hipSuccess ||
      (e = hipMalloc(&P->d_start3, sizeof(int) * (P->grid3 + 1))) != hipSuccess) {
    hard_batch_plan_destroy(P);
    return hip_fail(e, "hard_batch_plan_create alloc");
  }
  if ((e = hipMemcpy(P->d_probs, probs.data(), sizeof(BatchProblem) * nprob, hipMemcpyHostToDevice)) != hipSuccess ||
      (P->nitems12 && (e = hipMemcpy(P->d_items12, i12.data(), sizeof(WorkItem) * P->nitems12, hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->nitems3 && (e = hipMemcpy(P->d_items3, i3.data(), sizeof(WorkItem) * P->nitems3, hipMemcpyHostToDevice)) != hipSuccess) ||
      (e = hipMemcpy(P->d_start12, s12.data(), sizeof(int) * (P->grid12 + 1), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(P->d_start3, s3.data(), sizeof(int) * (P->grid3 + 1), hipMemcpyHostToDevice)) != hipSuccess) {
    hard_batch_plan_destroy(P);
    return hip_fail(e, "hard_batch_plan_create copy");
  }
  // workspace: control | run counter | slot[items] | t[nprob] | steps[nprob] |
  // stage state
  P->ws_ctl = 0;
  P->ws_active = 256;
  P->ws_slot = 512;
  P->ws_t = P->ws_slot + al256(sizeof(double) * (size_t)nslot);
  P->ws_steps = P->ws_t + al256(sizeof(double) * nprob);
  P->ws_stage = P->ws_steps + al256(sizeof(long long) * nprob);
  P->ws_total = P->ws_stage + al256((size_t)P->total_elems * P->wsize);
  *out = P;
  return ok();
}

hard_status_t hard_batch_plan_destroy(hard_batch_plan_t* P) {
  if (!P) return ok();
  if (P->d_probs) (void)hipFree(P->d_probs);
  if (P->d_items12) (void)hipFree(P->d_items12);
  if (P->d_items3) (void)hipFree(P->d_items3);
  if (P->d_start12) (void)hipFree(P->d_start12);
  if (P->d_start3) (void)hipFree(P->d_start3);
  delete P;
  return ok();
}

hard_status_t hard_batch_offsets(const hard_batch_plan_t* P, int64_t* offsets) {
  if (!P || !offsets) return fail(HARD_ERR_INVALID_ARG, "plan and offsets must not be NULL");
  std::memcpy(offsets, P->offsets.data(), sizeof(int64_t) * (P->nprob + 1));
  return ok();
}

hard_status_t hard_batch_workspace_bytes(const hard_batch_plan_t* P, size_t* bytes) {
  if (!P || !bytes) return fail(HARD_ERR_INVALID_ARG, "plan and bytes must not be NULL");
  *bytes = P->ws_total;
  return ok();
}

hard_status_t hard_cfl_dt_batched(const hard_batch_plan_t* P, const void* U, double cfl,
                                  double* dt_dev, void* work, size_t work_bytes, void* stream) {
  BatchArgs a;
  hard_status_t st = batch_common(P, U, dt_dev, work, work_bytes, &a);
  if (st) return st;
  if ((st = check_cfl(cfl))) return st;
  a.src = U;
  hipStream_t s = (hipStream_t)stream;
  const int TX3 = kTiles3D[P->tile3d][0], TY3 = kTiles3D[P->tile3d][1];
  if (P->nitems12) {
    BatchArgs b = a;
    b.items = P->d_items12;
    b.nitems = P->nitems12;
    if (P->dtype == HARD_F64)
      hipLaunchKernelGGL((batched_cfl<double, BT12>), dim3(P->grid12), dim3(BT12), 0, s, b, TX3, TY3);
    else
      hipLaunchKernelGGL((batched_cfl<float, BT12>), dim3(P->grid12), dim3(BT12), 0, s, b, TX3, TY3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "hard_cfl_dt_batched");
  }
  if (P->nitems3) {
    BatchArgs b = a;
    b.items = P->d_items3;
    b.nitems = P->nitems3;
    if (P->dtype == HARD_F64)
      hipLaunchKernelGGL((batched_cfl<double, BT3>), dim3(P->grid3), dim3(BT3), 0, s, b, TX3, TY3);
    else
      hipLaunchKernelGGL((batched_cfl<float, BT3>), dim3(P->grid3), dim3(BT3), 0, s, b, TX3, TY3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "hard_cfl_dt_batched");
  }
  hipError_t e = launch_dt_final(P, a, cfl, s);
  if (e != hipSuccess) return hip_fail(e, "hard_cfl_dt_batched final");
  return ok();
}

hard_status_t hard_hydro_step_batched(const hard_batch_plan_t* P, void* U, double* dt_dev,
                                      double cfl, int32_t update_dt, void* work,
                                      size_t work_bytes, void* stream) {
  BatchArgs a;
  hard_status_t st = batch_common(P, U, dt_dev, work, work_bytes, &a);
  if (st) return st;
  if (update_dt && (st = check_cfl(cfl))) return st;
  char* wb = static_cast<char*>(work);
  void* U1 = wb + P->ws_stage;
  hipStream_t s = (hipStream_t)stream;
  a.fuse_cfl = 0;
  a.src = U;
  a.un = U;
  a.dst = U1;
  hipError_t e = P->dtype == HARD_F64 ? launch_batched_stage<double, 1>(P, a, wb, s)
                                      : launch_batched_stage<float, 1>(P, a, wb, s);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step_batched stage 1");
  a.src = U1;
  a.un = U;
  a.dst = U;
  a.fuse_cfl = update_dt ? 1 : 0;
  e = P->dtype == HARD_F64 ? launch_batched_stage<double, 2>(P, a, wb, s)
                           : launch_batched_stage<float, 2>(P, a, wb, s);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step_batched stage 2");
  if (update_dt && (e = launch_dt_final(P, a, cfl, s)) != hipSuccess)
    return hip_fail(e, "hard_hydro_step_batched dt");
  return ok();
}

hard_status_t hard_run_batched(const hard_batch_plan_t* P, void* U, double cfl, double t_end,
                               int64_t max_steps, double* dt_dev, double* t_host,
                               int64_t* steps_host, void* work, size_t work_bytes, void* stream) {
  BatchArgs a;
  hard_status_t st = batch_common(P, U, dt_dev, work, work_bytes, &a);
  if (st) return st;
  if ((st = check_cfl(cfl))) return st;
  if (!(std::isfinite(t_end) && t_end > 0.0)) return fail(HARD_ERR_INVALID_ARG, "t_end must be finite and > 0");
  if (max_steps < 1) return fail(HARD_ERR_INVALID_ARG, "max_steps must be >= 1");
  char* wb = static_cast<char*>(work);
  hipStream_t s = (hipStream_t)stream;
  double* t = reinterpret_cast<double*>(wb + P->ws_t);
  long long* steps = reinterpret_cast<long long*>(wb + P->ws_steps);
  unsigned* active = reinterpret_cast<unsigned*>(wb + P->ws_active);
  const int nb = (P->nprob + 255) / 256;
  hipLaunchKernelGGL(batched_run_clear, dim3(nb), dim3(256), 0, s, P->nprob, t, steps, active);
  if ((st = hard_cfl_dt_batched(P, U, cfl, dt_dev, work, work_bytes, stream))) return st;
  const int batch = 32;
  for (;;) {
    hipLaunchKernelGGL(counter_clear, dim3(1), dim3(64), 0, s, active);
    for (int i = 0; i < batch; ++i) {
      hipLaunchKernelGGL(batched_time_control, dim3(nb), dim3(256), 0, s, P->nprob, dt_dev, t, steps,
                         t_end, (long long)max_steps, active);
      if ((st = hard_hydro_step_batched(P, U, dt_dev, cfl, 1, work, work_bytes, stream))) return st;
    }
    hipError_t e;
    unsigned act = 0;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_run_batched sync");
    if ((e = hipMemcpy(&act, active, sizeof act, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hard_run_batched read");
    if (act == 0) break;
  }
  hipError_t e;
  unsigned flags = 0;
  if ((t_host && (e = hipMemcpy(t_host, t, sizeof(double) * P->nprob, hipMemcpyDeviceToHost)) != hipSuccess) ||
      (steps_host && (e = hipMemcpy(steps_host, steps, sizeof(long long) * P->nprob, hipMemcpyDeviceToHost)) != hipSuccess) ||
      (e = hipMemcpy(&flags, &a.ctl->flags, sizeof flags, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hard_run_batched read");
  if (flags) return fail(HARD_ERR_NONPHYSICAL, "non-physical state (flags 0x%x)", flags);
  return ok();
}

}  // extern "C"
