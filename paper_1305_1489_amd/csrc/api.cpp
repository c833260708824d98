// Host-side entry points of libhdg that launch no kernels: error reporting, the
// discretisation handle (reference tables), and host-side checks.
#include <cstring>
#include <string>
#include <vector>

#include "hdg_internal.h"

namespace hdg {

static thread_local std::string g_last_error = "no error";

hdg_status set_error(hdg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

hdg_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return HDG_OK;
  return set_error(HDG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Kernel timer of hdg_set_kernel_timer (per thread, like the error message).
static thread_local std::string g_timer_kernel;
static thread_local hipEvent_t g_timer_start = nullptr, g_timer_stop = nullptr;

void timer_begin(const char* kernel, hipStream_t s) {
  if (g_timer_start && g_timer_kernel == kernel) (void)hipEventRecord(g_timer_start, s);
}
void timer_end(const char* kernel, hipStream_t s) {
  if (g_timer_stop && g_timer_kernel == kernel) (void)hipEventRecord(g_timer_stop, s);
}

}  // namespace hdg

using namespace hdg;

extern "C" {

const char* hdg_last_error(void) { return g_last_error.c_str(); }

int hdg_max_degree(void) { return kMaxDegree; }

hdg_status hdg_set_kernel_timer(const char* kernel, void* ev_start, void* ev_stop) {
  if (!kernel) {
    g_timer_kernel.clear();
    g_timer_start = g_timer_stop = nullptr;
    return HDG_OK;
  }
  if (!ev_start || !ev_stop) return set_error(HDG_ERR_INVALID_ARG, "hdg_set_kernel_timer: NULL event");
  g_timer_kernel = kernel;
  g_timer_start = (hipEvent_t)ev_start;
  g_timer_stop = (hipEvent_t)ev_stop;
  return HDG_OK;
}

// Launch shapes of the single-mesh condensation, per degree (persistent grids; the tile
// kernels of k = 1..3 run four elements per wavefront, so waves_per_element is 1).
// Degrees 5 and 6 use workgroups_per_cu and xcd_remap only (four wavefronts per element at
// k = 5, six at k = 6).
static hdg_tile_config g_launch[kMaxDegree + 1] = {{2, 0, 1}, {4, 1, 1}, {4, 1, 1}, {4, 1, 1}, {2, 1, 4},
                                                   {1, 0, 4}, {1, 0, 4}};

hdg_status hdg_set_launch_config(int k, const hdg_tile_config* cfg) {
  if (k < 0 || k > kMaxDegree || !cfg) return set_error(HDG_ERR_INVALID_ARG, "hdg_set_launch_config: bad argument");
  const bool tile = k >= 1 && k <= 3;
  const int w = cfg->waves_per_element;
  if (cfg->workgroups_per_cu < 1 || cfg->workgroups_per_cu > 64 || (cfg->xcd_remap != 0 && cfg->xcd_remap != 1) ||
      (tile ? w != 1 : (w != 1 && w != 2 && w != 4 && w != 8)))
    return set_error(HDG_ERR_INVALID_ARG, "hdg_set_launch_config: shape out of range");
  g_launch[k] = *cfg;
  return HDG_OK;
}

hdg_status hdg_get_launch_config(int k, hdg_tile_config* cfg) {
  if (k < 0 || k > kMaxDegree || !cfg) return set_error(HDG_ERR_INVALID_ARG, "hdg_get_launch_config: bad argument");
  *cfg = g_launch[k];
  return HDG_OK;
}

hdg_status hdg_disc_create(int k, int nq, hdg_disc** out) {
  if (!out) return set_error(HDG_ERR_INVALID_ARG, "hdg_disc_create: out is NULL");
  *out = nullptr;
  if (k < 0 || k > kMaxDegree)
    return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_disc_create: degree must be in 0.." + std::to_string(kMaxDegree));
  if (nq == 0) nq = k + 2;
  if (nq < k + 1 || nq > 8) return set_error(HDG_ERR_INVALID_ARG, "hdg_disc_create: nq must be in k+1..8");
  hdg_disc* d = new hdg_disc();
  try {
    d->host = build_tables(k, nq);
  } catch (const std::exception& ex) {
    delete d;
    return set_error(HDG_ERR_INVALID_ARG, std::string("hdg_disc_create: ") + ex.what());
  }
  const auto& h = d->host;
  hipError_t e = hipMalloc(&d->d_tables, sizeof(double) * h.data.size());
  if (e != hipSuccess) {
    delete d;
    return check_hip(e, "hdg_disc_create: hipMalloc");
  }
  e = hipMemcpy(d->d_tables, h.data.data(), sizeof(double) * h.data.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d->d_tables);
    delete d;
    return check_hip(e, "hdg_disc_create: hipMemcpy");
  }
  const auto& o = h.off;
  const double* b = d->d_tables;
  d->dev = Tables{b + o.vol_w, b + o.lambda, b + o.P, b + o.Pg, b + o.tri_w, b + o.xi, b + o.D,
                  b + o.Chat, b + o.PP, b + o.DP, b + o.P1g, b + o.Shat, b + o.Pt, b + o.ChatT,
                  b + o.PPt, b + o.DPT, b + o.P1gt, b + o.Shatt, b + o.DPtopinv, b + o.Pface, b + o.Dmu,
                  b + o.tri_pts};
  d->factor_len = tile_factor_len(k) ? tile_factor_len(k) : h.d3 * (h.d3 + 1) + h.d3;
  *out = d;
  return HDG_OK;
}

hdg_status hdg_disc_destroy(hdg_disc* disc) {
  if (!disc) return HDG_OK;
  hipError_t e = disc->d_tables ? hipFree(disc->d_tables) : hipSuccess;
  delete disc;
  return check_hip(e, "hdg_disc_destroy: hipFree");
}

hdg_status hdg_disc_get_info(const hdg_disc* disc, hdg_disc_info* info) {
  if (!disc || !info) return set_error(HDG_ERR_INVALID_ARG, "hdg_disc_get_info: NULL argument");
  const auto& h = disc->host;
  info->k = h.k;
  info->nq = h.nq;
  info->d3 = h.d3;
  info->d2 = h.d2;
  info->m = 4 * h.d2;
  info->d3p = h.d3p;
  info->nqd = h.nqd;
  info->nqd2 = h.nqd2;
  info->factor_len = disc->factor_len;
  return HDG_OK;
}

static hdg_status table_lookup(const HostTables& h, const char* name, double* h_out, int64_t* count) {
  const auto& o = h.off;
  struct Ent {
    const char* n;
    int off, len;
  } ents[] = {
      {"vol_pts", o.vol_pts, 3 * h.nqd},      {"vol_w", o.vol_w, h.nqd},
      {"tri_pts", o.tri_pts, 2 * h.nqd2},     {"tri_w", o.tri_w, h.nqd2},
      {"P", o.P, h.nqd * h.d3},               {"Pgrad", o.Pg, 3 * h.nqd * h.d3},
      {"D", o.D, h.nqd2 * h.d2},              {"Pface", o.Pface, 4 * h.nqd2 * h.d3},
      {"Chat", o.Chat, 3 * h.d3 * h.d3},      {"PP", o.PP, 4 * h.d3 * h.d3},
      {"DP", o.DP, 24 * h.d2 * h.d3},         {"P1grad", o.P1g, 3 * h.nqd * h.d3p},
      {"Shat", o.Shat, 6 * h.d3p * h.d3p},    {"DPtopinv", o.DPtopinv, 24 * h.d2 * h.d2},
      {"Dmu", o.Dmu, 6 * h.nqd2 * h.d2},
      {"P1grad_pad", o.P1gt, 3 * h.nqp * h.d3pp4},
      {"Shat_tiles", o.Shatt, 6 * (h.d3pp4 / 4) * (h.d3pp4 / 4 + 1) / 2 * 16},
  };
  for (const auto& e : ents) {
    if (std::strcmp(e.n, name) == 0) {
      *count = e.len;
      if (h_out) std::memcpy(h_out, h.data.data() + e.off, sizeof(double) * e.len);
      return HDG_OK;
    }
  }
  return set_error(HDG_ERR_INVALID_ARG, std::string("unknown table ") + name);
}

hdg_status hdg_disc_table(const hdg_disc* disc, const char* name, double* h_out, int64_t* count) {
  if (!disc || !name || !count) return set_error(HDG_ERR_INVALID_ARG, "hdg_disc_table: NULL argument");
  return table_lookup(disc->host, name, h_out, count);
}

hdg_status hdg_reference_table(int k, int nq, const char* name, double* h_out, int64_t* count) {
  if (!name || !count) return set_error(HDG_ERR_INVALID_ARG, "hdg_reference_table: NULL argument");
  if (k < 0 || k > kMaxDegree) return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_reference_table: degree");
  if (nq == 0) nq = k + 2;
  if (nq < k + 1 || nq > 8) return set_error(HDG_ERR_INVALID_ARG, "hdg_reference_table: nq must be in k+1..8");
  HostTables h = build_tables(k, nq);
  return table_lookup(h, name, h_out, count);
}

hdg_status hdg_check_tau(const hdg_mesh* mesh, const double* d_tau, void* stream) {
  if (!mesh || !d_tau) return set_error(HDG_ERR_INVALID_ARG, "hdg_check_tau: NULL argument");
  std::vector<double> t(4 * mesh->nelt);
  hipError_t e = hipMemcpyAsync(t.data(), d_tau, sizeof(double) * t.size(), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return check_hip(e, "hdg_check_tau");
  for (int64_t K = 0; K < mesh->nelt; ++K) {
    double mx = 0;
    for (int l = 0; l < 4; ++l) {
      double v = t[4 * K + l];
      if (!(v >= 0)) return set_error(HDG_ERR_TAU_ZERO, "tau is negative or NaN on element " + std::to_string(K));
      mx = v > mx ? v : mx;
    }
    if (mx == 0) return set_error(HDG_ERR_TAU_ZERO, "tau vanishes on every face of element " + std::to_string(K));
  }
  return HDG_OK;
}

}  // extern "C"

namespace hdg {

hdg_tile_config launch_config(int k) { return g_launch[k]; }

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace hdg
