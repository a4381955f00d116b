// Batched persistent execution of many interpolation jobs (flints_batch_*).
//
// Jobs are grouped by system-size class (row group n <= 16 / n <= 32, tile
// n <= 48 / n <= 64) and cut into tiles of consecutive targets (multiples of 64
// so fix-up chunks never straddle tiles).  One persistent launch per class:
// in the row-group classes every block takes the next tile from a device queue
// (an atomic counter) and reloads the job's correlation table into LDS when the
// job changes; in the tile classes, whose systems fill the LDS, the tables are
// read through the caches and every wave takes tiles on its own.  Both run the
// shared per-group / per-point bodies of device.h, so a target gets exactly the
// arithmetic of flints_interpolate.  Spin 0 and spin 2 jobs share a launch
// (both bodies are compiled into it).  A second persistent launch per class
// runs the fix-up pass over the same tiles.  The queue counters are cleared by
// a kernel at the start of every run, which keeps the sequence capturable in a
// HIP graph and its replays exact.
#include "device.h"
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

namespace flints {

struct BatchJob {
  PlanDev P;
  const double *map, *theta, *phi;
  double *out, *var;
  int64_t n;
};

struct BatchTile {
  int32_t job;
  int32_t pad;
  int64_t start, count;
};

constexpr int NENGINE = 4;   // row group NT = 1, 2; tile T = 3, 4
constexpr int NTABB = 6;     // table-size buckets: <= 16, 36, 57, 77, 98 KB, larger
constexpr int NCLASS = NENGINE * NTABB;   // launch groups, index NTABB * engine + bucket
static_assert(sizeof(flints_batch_info_t::tiles) / sizeof(int) == NCLASS,
              "flints_batch_info_t holds one entry per launch group");
static_assert(2 * NCLASS <= 64, "k_batch_reset clears the queue counters with one wave");

__global__ void k_batch_reset(unsigned *ctr, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ctr[i] = 0u;
}

template <int CLS, int SPIN>
__device__ inline void batch_tile_main(const BatchJob &J, const double *tab, const WaveBufs &B,
                                       const BatchTile &T, int wave, int wpb, int lane) {
  if constexpr (CLS < 2) {
    const int64_t ngroups = (T.count + 3) / 4;
    for (int64_t g = wave; g < ngroups; g += wpb)
      group_rs<CLS + 1, SPIN>(J.P, tab, J.map, J.theta, J.phi, J.n, J.out, J.var, B, T.start + 4 * g,
                              lane);
  } else {
    for (int64_t i = wave; i < T.count; i += wpb)
      point_tile<CLS + 1, SPIN>(J.P, tab, J.map, J.theta, J.phi, J.n, J.out, J.var, B, T.start + i,
                                lane);
  }
}

template <int CLS, int SPIN>
__device__ inline void batch_tile_fixup(const BatchJob &J, const double *tab, const WaveBufs &B,
                                        const BatchTile &T, int wave, int wpb, int lane) {
  const int64_t nch = (T.count + WAVE - 1) / WAVE;
  for (int64_t c = wave; c < nch; c += wpb) {
    if constexpr (CLS < 2)
      fixup_chunk<RowGroupEngine<CLS + 1, SPIN>, SPIN>(J.P, tab, J.map, J.theta, J.phi, J.n, J.out,
                                                       J.var, B, T.start + c * WAVE, lane);
    else
      fixup_chunk<TileEngine<CLS + 1, SPIN>, SPIN>(J.P, tab, J.map, J.theta, J.phi, J.n, J.out,
                                                   J.var, B, T.start + c * WAVE, lane);
  }
}

// Persistent launch over the class's tile queue (FIX selects the fix-up pass).
// Tile classes read their tables through the caches, so each wave takes tiles
// on its own (no block barriers); row-group classes copy the job's table to
// LDS, so a block takes a tile and shares it among its waves.
template <int CLS, bool FIX>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_batch(const BatchJob *__restrict__ jobs,
                                               const BatchTile *__restrict__ tiles, int ntiles,
                                               unsigned *ctr, Layout L) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_tile;
  char *lds = (char *)lds_dyn;
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  if constexpr (CLS >= 2) {
    for (;;) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(ctr, 1u);
      t = __shfl(t, 0);
      if (t >= ntiles) break;
      const BatchTile T = tiles[t];
      const BatchJob &J = jobs[T.job];
      if (J.P.spin == 0) {
        if (FIX) batch_tile_fixup<CLS, 0>(J, J.P.tab, B, T, 0, 1, lane);
        else batch_tile_main<CLS, 0>(J, J.P.tab, B, T, 0, 1, lane);
      } else {
        if (FIX) batch_tile_fixup<CLS, 2>(J, J.P.tab, B, T, 0, 1, lane);
        else batch_tile_main<CLS, 2>(J, J.P.tab, B, T, 0, 1, lane);
      }
    }
    return;
  }
  int cur = -1;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(ctr, 1u);
    __syncthreads();
    const int t = s_tile;
    __syncthreads();   // every thread has read s_tile before it is overwritten
    if (t >= ntiles) break;
    const BatchTile T = tiles[t];
    const BatchJob &J = jobs[T.job];
    if (T.job != cur) {
      const int nt = J.P.ntab * J.P.nfun;
      for (int i = threadIdx.x; i < nt; i += blockDim.x) ((double *)lds)[i] = J.P.tab[i];
      __syncthreads();
      cur = T.job;
    }
    const double *tab = (const double *)lds;
    if (J.P.spin == 0) {
      if (FIX) batch_tile_fixup<CLS, 0>(J, tab, B, T, wave, wpb, lane);
      else batch_tile_main<CLS, 0>(J, tab, B, T, wave, wpb, lane);
    } else {
      if (FIX) batch_tile_fixup<CLS, 2>(J, tab, B, T, wave, wpb, lane);
      else batch_tile_main<CLS, 2>(J, tab, B, T, wave, wpb, lane);
    }
    __syncthreads();   // the tile is finished before the table may be replaced
  }
}

// ---------------------------------------------------------------- host side

struct ClassRun {
  int used = 0;
  int max_K = 0, max_n = 0, max_tab = 0;
  int tile_pts = 4096;   // targets per tile (tile classes: per wave, set at creation)
  int wpb = 0, occ = 1, lds = 0;
  Layout L{};
  BatchTile *d_tiles = nullptr;
  int ntiles = 0;
};

struct Batch {
  int device = 0;
  std::vector<flints_job_t> jobs;
  std::vector<int> cls;        // class per job, -1 = single-plan path, -2 = empty
  BatchJob *d_jobs = nullptr;
  unsigned *d_ctr = nullptr;   // [2 * NCLASS]: main and fix-up queue per class
  ClassRun run[NCLASS];
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t points = 0;
};

// Launch group of a job: engine by system size, and for the row-group engines
// (which copy the table to LDS) a table-size bucket, so that a large table does
// not set the occupancy of jobs with small ones.  The tile engines read the
// table through the caches, so each is one launch group whatever the tables.
static int job_class(const Plan *p) {
  if (p->d.precision != FLINTS_FP64 || p->d.var_kind != FLINTS_VAR_PAPER) return -1;
  if (p->d.stencil_mode != FLINTS_STENCIL_NEAREST) return -1;   // tabulated stencils: own kernel
  const int n = p->d.n;
  if (n > 64) return -1;   // the LDS elimination runs through the single-plan path
  const int e = n <= 16 ? 0 : n <= 32 ? 1 : n <= 48 ? 2 : 3;
  if (e >= 2) return NTABB * e;
  const int tb = p->d.ntab * p->d.nfun * 8;
  static const int edge_kb[NTABB - 1] = {16, 36, 57, 77, 98};
  int k = 0;
  while (k < NTABB - 1 && tb > (edge_kb[k] << 10)) ++k;
  return NTABB * e + k;
}

template <int CLS, bool FIX>
static const void *batch_kernel() {
  return (const void *)k_batch<CLS, FIX>;
}

static const void *class_kernel(int c, bool fix) {
  switch (c / NTABB) {
    case 0: return fix ? batch_kernel<0, true>() : batch_kernel<0, false>();
    case 1: return fix ? batch_kernel<1, true>() : batch_kernel<1, false>();
    case 2: return fix ? batch_kernel<2, true>() : batch_kernel<2, false>();
    default: return fix ? batch_kernel<3, true>() : batch_kernel<3, false>();
  }
}

static void launch_class(int c, bool fix, int blocks, int wpb, int lds, hipStream_t s,
                         const BatchJob *jobs, const BatchTile *tiles, int ntiles, unsigned *ctr,
                         const Layout &L) {
  const dim3 g((unsigned)blocks), b((unsigned)(wpb * WAVE));
  switch (c / NTABB) {
    case 0:
      if (fix) hipLaunchKernelGGL((k_batch<0, true>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      else hipLaunchKernelGGL((k_batch<0, false>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      break;
    case 1:
      if (fix) hipLaunchKernelGGL((k_batch<1, true>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      else hipLaunchKernelGGL((k_batch<1, false>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      break;
    case 2:
      if (fix) hipLaunchKernelGGL((k_batch<2, true>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      else hipLaunchKernelGGL((k_batch<2, false>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      break;
    default:
      if (fix) hipLaunchKernelGGL((k_batch<3, true>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      else hipLaunchKernelGGL((k_batch<3, false>), g, b, lds, s, jobs, tiles, ntiles, ctr, L);
      break;
  }
}

// Tiles of `tile_pts` targets (a multiple of 64) over the first `limit`
// targets of every job of class c (limit < 0: all targets).
static std::vector<BatchTile> make_tiles(const Batch &b, int c, int tile_pts, int64_t limit) {
  std::vector<BatchTile> t;
  for (size_t j = 0; j < b.jobs.size(); ++j) {
    if (b.cls[j] != c) continue;
    const int64_t n = limit < 0 ? b.jobs[j].n : std::min<int64_t>(b.jobs[j].n, limit);
    for (int64_t s = 0; s < n; s += tile_pts) {
      BatchTile bt;
      bt.job = (int32_t)j;
      bt.pad = 0;
      bt.start = s;
      bt.count = std::min<int64_t>(tile_pts, n - s);
      t.push_back(bt);
    }
  }
  return t;
}

// LDS layout and the waves-per-block choice (most waves per CU) for class c.
static int size_class(ClassRun &r, int c, int wpb_cap) {
  const int e = c / NTABB;
  const int ppw = e < 2 ? 4 : 1;
  const int min_mat = e < 2 ? 0 : e * TILE_D + 16;   // tile path T = e + 1: T - 1 staged tiles + pivots
  r.L = make_layout(r.max_tab, 1, r.max_K, r.max_n, ppw, 1, 3, min_mat);
  // tile classes read the job's table through the caches: their systems fill
  // the LDS, and a table copy beside them would cost waves
  if (e >= 2) r.L.tab_bytes = 0;
  int lds_max = 0, ncu = 0, dev = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const void *km = class_kernel(c, false);
  int best = 0;
  r.wpb = 0;
  for (int w = 1; w <= std::min(MAX_WPB, wpb_cap); ++w) {
    const int l = r.L.tab_bytes + w * r.L.wave_bytes;
    if (l + 64 > lds_max) break;   // room for the kernel's static queue slot
    hipFuncSetAttribute(km, hipFuncAttributeMaxDynamicSharedMemorySize, l);
    int o = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, km, w * WAVE, l);
    if (o * w >= best && o > 0) { best = o * w; r.wpb = w; r.occ = o; }
  }
  if (r.wpb == 0) {
    set_error("batch class needs more LDS than the device offers");
    return FLINTS_ELIMIT;
  }
  r.lds = r.L.tab_bytes + r.wpb * r.L.wave_bytes;
  hipFuncSetAttribute(km, hipFuncAttributeMaxDynamicSharedMemorySize, r.lds);
  hipFuncSetAttribute(class_kernel(c, true), hipFuncAttributeMaxDynamicSharedMemorySize, r.lds);
  return FLINTS_OK;
}

static int grid_blocks(const ClassRun &r) {
  int ncu = 0, dev = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  return std::max(1, std::min(r.ntiles, ncu * r.occ));
}

static int enqueue(Batch *b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b->d_ctr, 2 * NCLASS);
  for (int c = 0; c < NCLASS; ++c) {
    ClassRun &r = b->run[c];
    if (!r.used || r.ntiles == 0) continue;
    const int blocks = grid_blocks(r);
    launch_class(c, false, blocks, r.wpb, r.lds, s, b->d_jobs, r.d_tiles, r.ntiles, b->d_ctr + 2 * c, r.L);
    launch_class(c, true, blocks, r.wpb, r.lds, s, b->d_jobs, r.d_tiles, r.ntiles,
                 b->d_ctr + 2 * c + 1, r.L);
  }
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    if (b->cls[j] != -1) continue;
    const flints_job_t &jb = b->jobs[j];
    const Plan *p = reinterpret_cast<const Plan *>(jb.plan);
    const int rc = launch_interpolate(p, (const double *)jb.map, jb.theta, jb.phi, jb.n,
                                      (double *)jb.out, (double *)jb.var, s);
    if (rc != FLINTS_OK) return rc;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("batch launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

// Host-to-device upload on a private non-blocking stream of default priority,
// so that creating a batch does not wait for work in flight on other streams
// (a plain hipMemcpy runs on the null stream).
static bool upload(void *dst, const void *src, size_t bytes) {
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return false;
  const bool ok = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess &&
                  hipStreamSynchronize(st) == hipSuccess;
  (void)hipStreamDestroy(st);
  return ok;
}

// Time one class's main pass over a sample of the batch for a candidate tile
// size and waves-per-block cap; returns seconds (or a large value on failure).
static double time_candidate(Batch *b, int c, int tile_pts, int wpb_cap, int64_t limit) {
  ClassRun r = b->run[c];
  r.tile_pts = tile_pts;
  if (size_class(r, c, wpb_cap) != FLINTS_OK) return 1e30;
  std::vector<BatchTile> t = make_tiles(*b, c, tile_pts, limit);
  if (t.empty()) return 1e30;
  BatchTile *d_t = nullptr;
  if (hipMalloc(&d_t, t.size() * sizeof(BatchTile)) != hipSuccess) return 1e30;
  hipMemcpy(d_t, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  r.ntiles = (int)t.size();
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double best = 1e30;
  for (int rep = 0; rep < 2; ++rep) {   // first repetition warms caches and code
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, nullptr, b->d_ctr, 2 * NCLASS);
    hipEventRecord(e0, nullptr);
    launch_class(c, false, grid_blocks(r), r.wpb, r.lds, nullptr, b->d_jobs, d_t, r.ntiles,
                 b->d_ctr + 2 * c, r.L);
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0) best = std::min(best, (double)ms * 1e-3);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(d_t);
  return best;
}

// Autotuner: tile sizes x waves-per-block caps, timed on the first
// `sample` targets of every job of the class; the fastest is kept.
constexpr int WAVE_TILE_PTS = 128;   // default tile of the tile classes (taken by one wave)

static void autotune(Batch *b, int c) {
  static const int block_tiles[] = {256, 1024, 4096, 16384};
  static const int wave_tiles[] = {64, 128, 256, 1024};
  const int *tiles = c / NTABB >= 2 ? wave_tiles : block_tiles;
  static const int caps[] = {MAX_WPB, 4, 2};
  int64_t cls_pts = 0, njobs = 0;
  for (size_t j = 0; j < b->jobs.size(); ++j)
    if (b->cls[j] == c) { cls_pts += b->jobs[j].n; ++njobs; }
  const int64_t sample = std::max<int64_t>(16384, (1 << 18) / std::max<int64_t>(njobs, 1));
  double best = 1e30;
  int bt = b->run[c].tile_pts, bw = MAX_WPB;
  for (int ti = 0; ti < 4; ++ti)
    for (int cap : caps) {
      const int tp = tiles[ti];
      const double t = time_candidate(b, c, tp, cap, sample);
      if (t < best) { best = t; bt = tp; bw = cap; }
    }
  b->run[c].tile_pts = bt;
  size_class(b->run[c], c, bw);
  (void)cls_pts;
}

static void free_batch(Batch *b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (auto &r : b->run)
    if (r.d_tiles) hipFree(r.d_tiles);
  if (b->d_jobs) hipFree(b->d_jobs);
  if (b->d_ctr) hipFree(b->d_ctr);
  delete b;
}

}  // namespace flints

using namespace flints;

extern "C" {

flints_batch_t flints_batch_create(const flints_job_t *jobs, int njobs, int flags) {
  if (!jobs || njobs < 1 || njobs > 65536) {
    set_error("jobs must be non-NULL and 1 <= njobs <= 65536");
    return nullptr;
  }
  Batch *b = new Batch();
  hipGetDevice(&b->device);
  b->jobs.assign(jobs, jobs + njobs);
  b->cls.assign(njobs, -2);
  std::vector<BatchJob> hj(njobs);
  for (int j = 0; j < njobs; ++j) {
    const flints_job_t &jb = jobs[j];
    if (!jb.plan || jb.n < 0 || (jb.n > 0 && (!jb.map || !jb.theta || !jb.phi || !jb.out))) {
      set_error("job " + std::to_string(j) + ": plan, map, theta, phi and out must be set and n >= 0");
      free_batch(b);
      return nullptr;
    }
    const Plan *p = reinterpret_cast<const Plan *>(jb.plan);
    if (p->device != b->device) {
      set_error("job " + std::to_string(j) + ": plan lives on another device");
      free_batch(b);
      return nullptr;
    }
    b->points += jb.n;
    hj[j].P = p->d;
    hj[j].map = (const double *)jb.map;
    hj[j].theta = jb.theta;
    hj[j].phi = jb.phi;
    hj[j].out = (double *)jb.out;
    hj[j].var = (double *)jb.var;
    hj[j].n = jb.n;
    if (jb.n == 0) continue;
    const int c = job_class(p);
    b->cls[j] = c;
    if (c < 0) continue;
    ClassRun &r = b->run[c];
    r.used = 1;
    r.max_K = std::max(r.max_K, p->d.K);
    r.max_n = std::max(r.max_n, p->d.n);
    r.max_tab = std::max(r.max_tab, p->d.ntab * p->d.nfun);
  }
  if (hipMalloc(&b->d_jobs, sizeof(BatchJob) * njobs) != hipSuccess ||
      hipMalloc(&b->d_ctr, sizeof(unsigned) * 2 * NCLASS) != hipSuccess) {
    set_error("device allocation for the batch failed");
    free_batch(b);
    return nullptr;
  }
  if (!upload(b->d_jobs, hj.data(), sizeof(BatchJob) * njobs)) {
    set_error("upload of the batch job table failed");
    free_batch(b);
    return nullptr;
  }
  for (int c = 0; c < NCLASS; ++c) {
    ClassRun &r = b->run[c];
    if (!r.used) continue;
    if (c / NTABB >= 2) r.tile_pts = WAVE_TILE_PTS;
    if (size_class(r, c, MAX_WPB) != FLINTS_OK) { free_batch(b); return nullptr; }
    if (flags & FLINTS_BATCH_AUTOTUNE) autotune(b, c);
    std::vector<BatchTile> t = make_tiles(*b, c, r.tile_pts, -1);
    r.ntiles = (int)t.size();
    if (hipMalloc(&r.d_tiles, sizeof(BatchTile) * std::max<size_t>(t.size(), 1)) != hipSuccess) {
      set_error("device allocation for the tile list failed");
      free_batch(b);
      return nullptr;
    }
    if (!t.empty() && !upload(r.d_tiles, t.data(), sizeof(BatchTile) * t.size())) {
      set_error("upload of the tile list failed");
      free_batch(b);
      return nullptr;
    }
  }
  if (hipGetLastError() != hipSuccess) {
    set_error("batch set-up failed on the device");
    free_batch(b);
    return nullptr;
  }
  return reinterpret_cast<flints_batch_t>(b);
}

int flints_batch_run(flints_batch_t batch, void *stream) {
  (void)hipGetLastError();   // errors of earlier calls are not this call's
  if (!batch) { set_error("batch is NULL"); return FLINTS_EINVAL; }
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (b->exec) {
    if (hipGraphLaunch(b->exec, (hipStream_t)stream) != hipSuccess) {
      set_error("graph launch failed");
      return FLINTS_EDEVICE;
    }
    return FLINTS_OK;
  }
  return enqueue(b, (hipStream_t)stream);
}

int flints_batch_capture(flints_batch_t batch, void *stream) {
  (void)hipGetLastError();   // errors of earlier calls are not this call's
  if (!batch) { set_error("batch is NULL"); return FLINTS_EINVAL; }
  Batch *b = reinterpret_cast<Batch *>(batch);
  hipStream_t s = (hipStream_t)stream;
  if (!s) { set_error("capture needs a non-null stream"); return FLINTS_EINVAL; }
  if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("hipStreamBeginCapture failed");
    return FLINTS_EDEVICE;
  }
  const int rc = enqueue(b, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != FLINTS_OK) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess || !g) { set_error("hipStreamEndCapture failed"); return FLINTS_EDEVICE; }
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    set_error("hipGraphInstantiate failed");
    return FLINTS_EDEVICE;
  }
  b->graph = g;
  return FLINTS_OK;
}

int flints_batch_info(flints_batch_t batch, flints_batch_info_t *info) {
  if (!batch || !info) { set_error("batch and info must be non-NULL"); return FLINTS_EINVAL; }
  const Batch *b = reinterpret_cast<const Batch *>(batch);
  std::memset(info, 0, sizeof(*info));
  info->njobs = (int)b->jobs.size();
  info->points = b->points;
  for (size_t j = 0; j < b->jobs.size(); ++j) info->fused_jobs += b->cls[j] >= 0;
  for (int c = 0; c < NCLASS; ++c) {
    const ClassRun &r = b->run[c];
    if (!r.used) continue;
    info->classes += 1;
    info->tiles[c] = r.ntiles;
    info->tile_points[c] = r.tile_pts;
    info->waves_per_block[c] = r.wpb;
  }
  info->captured = b->exec != nullptr;
  return FLINTS_OK;
}

void flints_batch_destroy(flints_batch_t batch) {
  if (!batch) return;
  free_batch(reinterpret_cast<Batch *>(batch));
}

}  // extern "C"
