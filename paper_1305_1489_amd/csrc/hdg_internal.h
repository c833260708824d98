// Internal declarations shared by the host and device sources of libhdg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdg.h"

namespace hdg {

constexpr int kMaxDegree = 6;
// Highest degree of the batched, FP32-refined and learned forms (the per-element LDS kernels).
constexpr int kMaxBatchDegree = 4;

inline constexpr int dim3(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }
inline constexpr int dim2(int k) { return (k + 1) * (k + 2) / 2; }
inline constexpr int tri(int n) { return n * (n + 1) / 2; }

// Offsets (in doubles) of every reference table inside the device table buffer.
// Doubles per element of the precomputed geometry record of the tile condensation (its
// workspace form): cofactors, det, |K|, normals, T_l, (n_l.n_m), perm, padding.
constexpr int kGeoRecord = 48;

// Doubles per (element, face) in the workspace of hdg_assemble_condense_ws: the upper
// triangle of the element's diagonal block of C^K (row-packed: row x holds columns x..d2-1)
// and its d2 entries of Cf^K.
constexpr int ws_block(int d2) { return d2 * (d2 + 1) / 2 + d2; }

// Byte layout of that workspace: the per-(element, face) contributions, then the geometry
// records, each 256-byte aligned.
inline size_t condense_ws_geo_offset(int d2, int64_t nelt) {
  return ((size_t)4 * nelt * ws_block(d2) * sizeof(double) + 255) / 256 * 256;
}
inline size_t condense_ws_bytes(int d2, int64_t nelt) {
  return condense_ws_geo_offset(d2, nelt) + (size_t)nelt * kGeoRecord * sizeof(double);
}

struct TableOffsets {
  int vol_pts, vol_w, lambda, P, Pg, tri_pts, tri_w, xi, D, Pface, Chat, PP, DP, P1g, Shat, DPtopinv, Dmu;
  // zero-padded copies for the 4x4-tile kernels (dimensions rounded up to multiples of 4)
  int Pt, ChatT, PPt, DPT;
  // for the postprocess kernel: degree k+1 gradients padded, stiffness tables as upper tiles
  int P1gt, Shatt;
  int total;
};

// Device view of the tables, passed to kernels by value.
struct Tables {
  const double* vol_w;   // [nqd]
  const double* lambda;  // [nqd][4]  barycentric coordinates of the volume points (eq 3.4)
  const double* P;       // [nqd][d3]  basis at the volume points (eq 3.5)
  const double* Pg;      // [3][nqd][d3] reference gradients (eq 3.66)
  const double* tri_w;   // [nqd2]
  const double* xi;      // [nqd2][3] barycentric coordinates of the face points (Section 4)
  const double* D;       // [nqd2][d2] face basis (eq 4.7)
  const double* Chat;    // [3][d3][d3] (eq 3.7)
  const double* PP;      // [4][d3][d3] (eq 4.5)
  const double* DP;      // [6][4][d2][d3] (eq 4.10)
  const double* P1g;     // [3][nqd][d3p] gradients of the degree k+1 basis
  const double* Shat;    // [6][d3p][d3p]
  const double* Pt;      // [nqp][d3p4]   P padded (nqp = nqd rounded up to 4, d3p4 = d3 rounded up)
  const double* ChatT;   // [3][d3p4][d3p4] transposes of Chat^h, padded
  const double* PPt;     // [4][d3p4][d3p4] PP_l padded
  const double* DPT;     // [6][4][d3p4][d2p4] transposes of DP_{mu,l}, padded
  const double* P1gt;    // [3][nqp][d3pp4]  P1g padded (d3pp4 = d3p rounded up to 4)
  const double* Shatt;   // [6][nus][16]  Shat as packed upper 4x4 tiles (nus = ts(ts+1)/2, ts = d3pp4/4)
  const double* DPtopinv;  // [6][4][d2][d2] inverse of DP_{mu,l}'s last d2 columns (eq 9.13)
  const double* Pface;  // [4][nqd2][d3] basis at the points of reference face l (eq 2.5)
  const double* Dmu;    // [6][nqd2][d2] face basis at F_mu(qhat_r) (eq 2.2)
  const double* tri_pts;  // [nqd2][2] face points (s, t) on the reference triangle
};

struct HostTables {
  int k, nq, d3, d2, d3p, nqd, nqd2;
  int d3p4, d2p4, nqp, d3pp4;  // padded sizes
  TableOffsets off;
  std::vector<double> data;
};

HostTables build_tables(int k, int nq);

// Doubles per element of the factor store of the tile kernels (0 where the degree uses
// the packed layout of the per-element kernel).
int tile_factor_len(int k);

// Device-side descriptor of one mesh of a batched condensation: the mesh, its coefficient
// arrays and its outputs, and the first work unit of the mesh in the degree's work list
// (a unit is a group of four elements for the tile kernels, one element otherwise).
struct BatchItem {
  hdg_mesh mesh;
  const double *kappa, *c, *f, *tau;
  double *H, *F, *factors;
  int unit_begin;
  int pad_;
};

// Degrees 5 and 6 (condense_big.hip): workspace bytes of the condensation of n elements,
// the condensation itself (ws: that workspace), and the postprocess u*.
size_t condense_big_workspace_bytes(int k, int64_t n);
hdg_status dispatch_condense_big(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                 const double* f, const double* tau, double* H, double* F, double* factors,
                                 const int* elems, int64_t n, double* Cout, double* Cfout, double* ws,
                                 size_t ws_bytes, hipStream_t s);
hdg_status launch_postprocess_big(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                                  const double* q, const double* u, double* us, hipStream_t s);

// Elements per work unit of the condensation kernel used for degree k.
int condense_unit(int k);

// Launch shape of the single-mesh condensation for degree k (hdg_set_launch_config).
hdg_tile_config launch_config(int k);
// Compute units of the current device (cached per device).
int device_cu_count();

// Persistent batched condensation of every mesh of degree k listed in d_items (device
// array, sorted by unit_begin); grid workgroups take the units round-robin, and with
// xcd_remap each of the eight XCDs takes a contiguous run of units per sweep.  waves is
// the number of wavefronts per element of the per-element kernel (k = 0, 4; 1, 2, 4 or 8).
hdg_status launch_batch_condense(int k, const Tables& tb, const BatchItem* d_items, int nitems, int total_units,
                                 int grid, int xcd_remap, int waves, hipStream_t s);

}  // namespace hdg

struct hdg_disc {
  hdg::HostTables host;
  double* d_tables = nullptr;
  hdg::Tables dev;
  int factor_len = 0;
};

namespace hdg {
hdg_status set_error(hdg_status s, const std::string& msg);
hdg_status check_hip(hipError_t e, const char* what);
// HDG_ERR_SINGULAR when the mesh has no Dirichlet face and c vanishes at every volume point
// (reads one device flag back: synchronises the stream, only in the no-Dirichlet case).
// hdg_set_kernel_timer: record the caller's events around the launch of the named kernel.
void timer_begin(const char* kernel, hipStream_t s);
void timer_end(const char* kernel, hipStream_t s);
hdg_status check_not_singular(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_c, hipStream_t s,
                              const char* who);
}  // namespace hdg

#define HDG_CHECK_LAUNCH(what)                                        \
  do {                                                                \
    hipError_t e__ = hipGetLastError();                               \
    if (e__ != hipSuccess) return hdg::check_hip(e__, what);          \
  } while (0)
