// Batched condensation of many independent meshes of mixed degree (the element work of
// Sections 3-6, eq 5.5-5.6 and the scatter of eq 6.5, for every mesh of the batch).
//
// Work list: per degree k, the meshes of that degree in the order given, each cut into
// work units (groups of four elements for the tile kernels of k = 1..3, single elements
// for k = 0 and 4).  One persistent kernel per degree sweeps its units; the per-element
// code is the same as in the single-mesh kernels, and the only cross-element writes
// (diagonal blocks of H and F) take at most two order-independent atomic adds, so every
// mesh's H, F and factors equal those of a separate hdg_assemble_condense bit for bit.
//
// A degree's part is: zero the diagonal blocks and F of its meshes, then the persistent
// condensation kernel.  The eager form runs the parts one after another (highest degree,
// i.e. the longest work, first); the captured form records the same chain as one hipGraph,
// replayed by one graph launch.  The parts are not run as parallel branches: each
// persistent kernel spreads its units statically over a grid sized for the whole chip,
// so a kernel sharing the compute units with another finishes with a long tail.
//
// The autotuner times, for one degree, every candidate launch shape on the batch itself
// and keeps the fastest: for the tile kernels the persistent grid size in {1, 2, 4, 8, 16}
// workgroups per compute unit, with and without the XCD-contiguous workgroup order; for
// the per-element kernel also the wavefronts per element in {1, 2, 4, 8} (its blocks fill
// most of the LDS, so at most one or two workgroups fit on a CU).
#include <algorithm>
#include <vector>

#include "device_common.h"

namespace hdg {

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

namespace {

__global__ void k_batch_zero(const BatchItem* __restrict__ items, int d2) {
  const BatchItem& it = items[blockIdx.y];
  const int64_t nfc = it.mesh.nfc;
  const int* __restrict__ diag = it.mesh.d_diag;
  const size_t bs = (size_t)d2 * d2, tot = (size_t)nfc * bs;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x) {
    const size_t f = i / bs, e = i % bs;
    it.H[(size_t)diag[f] * bs + e] = 0.0;
    if (e < (size_t)d2) it.F[f * d2 + e] = 0.0;
  }
}

}  // namespace
}  // namespace hdg

using namespace hdg;

struct hdg_batch {
  struct Degree {
    std::vector<BatchItem> items;
    BatchItem* d_items = nullptr;
    Tables tb{};
    int d2 = 0;
    int total_units = 0;
    int64_t nelt = 0;
    int64_t max_zero = 0;  // largest nfc * d2 * d2 of the degree's meshes
    hdg_tile_config cfg{0, 0, 1};
  };
  Degree deg[kMaxDegree + 1];
  int ncu = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(hdg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// The degree-k part (zero + persistent condensation) on stream s.
hdg_status run_degree(hdg_batch* b, int k, hipStream_t s) {
  auto& D = b->deg[k];
  if (D.items.empty()) return HDG_OK;
  const int nit = (int)D.items.size();
  const int64_t gx = std::min<int64_t>((D.max_zero + 255) / 256, 2048);
  if (gx > 0) {
    k_batch_zero<<<::dim3((unsigned)gx, (unsigned)nit), 256, 0, s>>>(D.d_items, D.d2);
    HDG_CHECK_LAUNCH("k_batch_zero");
  }
  const int64_t grid = std::min<int64_t>((int64_t)D.cfg.workgroups_per_cu * b->ncu, D.total_units);
  return launch_batch_condense(k, D.tb, D.d_items, nit, D.total_units, (int)std::max<int64_t>(grid, 1),
                               D.cfg.xcd_remap, D.cfg.waves_per_element, s);
}

hdg_status check_cfg(int k, const hdg_tile_config* c) {
  if (!c || c->workgroups_per_cu < 1 || c->workgroups_per_cu > 64 || (c->xcd_remap != 0 && c->xcd_remap != 1))
    return set_error(HDG_ERR_INVALID_ARG, "tile config: workgroups_per_cu must be 1..64 and xcd_remap 0 or 1");
  const int w = c->waves_per_element;
  if (condense_unit(k) == 4 ? w != 1 : (w != 1 && w != 2 && w != 4 && w != 8))
    return set_error(HDG_ERR_INVALID_ARG,
                     "tile config: waves_per_element must be 1 for k = 1..3 and 1, 2, 4 or 8 for k = 0, 4");
  return HDG_OK;
}

// Candidate shapes of the autotuner for degree k.
std::vector<hdg_tile_config> candidates(int k) {
  std::vector<hdg_tile_config> v;
  if (condense_unit(k) == 4) {
    for (int wpc : {1, 2, 4, 8, 16})
      for (int remap = 0; remap <= 1; ++remap) v.push_back({wpc, remap, 1});
  } else {
    for (int wpc : {1, 2})
      for (int remap = 0; remap <= 1; ++remap)
        for (int w : {1, 2, 4, 8}) v.push_back({wpc, remap, w});
  }
  return v;
}

}  // namespace

extern "C" hdg_status hdg_batch_create(int n, const hdg_batch_item* items, hdg_batch** out) {
  if (!out) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_create: out is NULL");
  *out = nullptr;
  if (n < 1 || !items) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_create: need n >= 1 items");
  for (int i = 0; i < n; ++i) {
    const hdg_batch_item& it = items[i];
    hdg_status st = check_disc_mesh(it.disc, it.mesh, "hdg_batch_create");
    if (st) return st;
    if (!it.d_kappa || !it.d_c || !it.d_f || !it.d_tau || !it.d_H || !it.d_F)
      return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_create: NULL array in item " + std::to_string(i));
    if (it.disc->host.k > kMaxBatchDegree)
      return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_batch_create: degrees 0..4 (item " + std::to_string(i) + ")");
    st = check_not_singular(it.disc, it.mesh, it.d_c, nullptr, "hdg_batch_create");
    if (st) return set_error(st, std::string(hdg_last_error()) + " (item " + std::to_string(i) + ")");
  }
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return check_hip(e, "hdg_batch_create: device query");
  hdg_batch* b = new hdg_batch();
  b->ncu = prop.multiProcessorCount;
  for (int i = 0; i < n; ++i) {
    const hdg_batch_item& it = items[i];
    const int k = it.disc->host.k;
    auto& D = b->deg[k];
    if (D.items.empty()) {
      D.tb = it.disc->dev;
      D.d2 = it.disc->host.d2;
      D.cfg = launch_config(k);
    }
    BatchItem bi{};
    bi.mesh = *it.mesh;
    bi.kappa = it.d_kappa;
    bi.c = it.d_c;
    bi.f = it.d_f;
    bi.tau = it.d_tau;
    bi.H = it.d_H;
    bi.F = it.d_F;
    bi.factors = it.d_factors;
    bi.unit_begin = D.total_units;
    const int64_t units = (it.mesh->nelt + condense_unit(k) - 1) / condense_unit(k);
    if (D.total_units + units > (int64_t)1 << 30 || D.items.size() >= 65535) {
      hdg_batch_destroy(b);
      return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_create: more than 65535 meshes or 2^30 work units of one degree");
    }
    D.total_units += (int)units;
    D.nelt += it.mesh->nelt;
    D.max_zero = std::max<int64_t>(D.max_zero, it.mesh->nfc * (int64_t)D.d2 * D.d2);
    D.items.push_back(bi);
  }
  e = hipSuccess;
  for (int k = 0; k <= kMaxDegree && e == hipSuccess; ++k) {
    auto& D = b->deg[k];
    if (D.items.empty()) continue;
    e = hipMalloc(&D.d_items, sizeof(BatchItem) * D.items.size());
    if (e == hipSuccess)
      e = hipMemcpy(D.d_items, D.items.data(), sizeof(BatchItem) * D.items.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    hdg_batch_destroy(b);
    return check_hip(e, "hdg_batch_create");
  }
  *out = b;
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_destroy(hdg_batch* b) {
  if (!b) return HDG_OK;
  drop_graph(b);
  hipError_t e = hipSuccess;
  for (auto& D : b->deg) {
    if (D.d_items) {
      hipError_t e2 = hipFree(D.d_items);
      if (e == hipSuccess) e = e2;
    }
  }
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return check_hip(e, "hdg_batch_destroy");
}

extern "C" hdg_status hdg_batch_info(const hdg_batch* b, int k, int64_t* nmesh, int64_t* nelt) {
  if (!b || k < 0 || k > kMaxDegree) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_info: bad argument");
  if (nmesh) *nmesh = (int64_t)b->deg[k].items.size();
  if (nelt) *nelt = b->deg[k].nelt;
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_set_config(hdg_batch* b, int k, const hdg_tile_config* cfg) {
  if (!b || k < 0 || k > kMaxDegree) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_set_config: bad argument");
  hdg_status st = check_cfg(k, cfg);
  if (st) return st;
  b->deg[k].cfg = *cfg;
  drop_graph(b);
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_get_config(const hdg_batch* b, int k, hdg_tile_config* cfg) {
  if (!b || !cfg || k < 0 || k > kMaxDegree)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_get_config: bad argument");
  *cfg = b->deg[k].cfg;
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_condense(hdg_batch* b, void* stream) {
  if (!b) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_condense: NULL batch");
  for (int k = kMaxDegree; k >= 0; --k) {
    hdg_status st = run_degree(b, k, (hipStream_t)stream);
    if (st) return st;
  }
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_capture(hdg_batch* b) {
  if (!b) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_capture: NULL batch");
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return check_hip(e, "hdg_batch_capture: begin");
  hdg_status st = HDG_OK;
  for (int k = kMaxDegree; k >= 0 && st == HDG_OK; --k)
    if (!b->deg[k].items.empty()) st = run_degree(b, k, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return check_hip(e, "hdg_batch_capture");
  }
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return check_hip(e, "hdg_batch_capture: instantiate");
  }
  return HDG_OK;
}

extern "C" hdg_status hdg_batch_launch(hdg_batch* b, void* stream) {
  if (!b) return set_error(HDG_ERR_INVALID_ARG, "hdg_batch_launch: NULL batch");
  if (!b->exec) {
    hdg_status st = hdg_batch_capture(b);
    if (st) return st;
  }
  return check_hip(hipGraphLaunch(b->exec, (hipStream_t)stream), "hdg_batch_launch");
}

extern "C" hdg_status hdg_autotune(hdg_batch* b, int k, int reps, hdg_tile_config* best, double* best_ms,
                                   int* ncand, hdg_tile_config* cands, double* cand_ms, void* stream) {
  if (!b || k < 0 || k > kMaxDegree || reps < 1)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_autotune: bad argument");
  auto& D = b->deg[k];
  if (D.items.empty()) return set_error(HDG_ERR_INVALID_ARG, "hdg_autotune: no mesh of this degree in the batch");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t t0, t1;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) return check_hip(e, "hdg_autotune: events");
  const hdg_tile_config saved = D.cfg;
  hdg_tile_config bc = saved;
  double bms = 1e300;
  int nc = 0;
  hdg_status st = HDG_OK;
  for (const hdg_tile_config& cand : candidates(k)) {
    {
      if (st || e != hipSuccess) break;
      D.cfg = cand;
      st = run_degree(b, k, s);  // warm-up
      if (st) break;
      e = hipEventRecord(t0, s);
      for (int r = 0; r < reps && st == HDG_OK && e == hipSuccess; ++r) st = run_degree(b, k, s);
      if (st || e != hipSuccess) break;
      e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e != hipSuccess) break;
      const double per = (double)ms / reps;
      if (cands) cands[nc] = D.cfg;
      if (cand_ms) cand_ms[nc] = per;
      ++nc;
      if (per < bms) {
        bms = per;
        bc = D.cfg;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st || e != hipSuccess) {
    D.cfg = saved;
    return st ? st : check_hip(e, "hdg_autotune");
  }
  D.cfg = bc;
  drop_graph(b);
  if (best) *best = bc;
  if (best_ms) *best_ms = bms;
  if (ncand) *ncand = nc;
  return HDG_OK;
}
