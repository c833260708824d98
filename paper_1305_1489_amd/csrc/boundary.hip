// Quadrature points in physical space and the boundary conditions of Section 6.
//   volume points  x_q = sum_i Lambda_{q i} v_i                          (eq 3.4)
//   face points    y_r = sum_i Xi_{r i} w_i in the face's own vertex order  (eq 6.2)
//   Dirichlet      uD_e = (v . D)^T u_D(y)       ((v . D)^T D = I for the orthonormal
//                  face basis, so eq 6.3 needs no solve)
//   Neumann        Phi_N = sum_s n_{e,s} (v . D)^T g_s(y)   (eq 6.4), added to F in a pass
//                  of its own after the scatter
//   elimination    (end of Section 6) Dirichlet rows become identity rows with right-hand
//                  side uD, and the Dirichlet columns of the free rows are moved to the
//                  right-hand side and zeroed, which keeps H symmetric positive definite.
#include <climits>

#include "device_common.h"

namespace hdg {
namespace {

template <int NQD>
__global__ void k_qp_coords(hdg_mesh mesh, const double* __restrict__ lambda, double* __restrict__ xyz) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)mesh.nelt * NQD) return;
  const int K = (int)(i / NQD), q = (int)(i % NQD);
  double x[3] = {0, 0, 0};
  for (int v = 0; v < 4; ++v) {
    const int id = mesh.d_elements[4 * K + v];
    const double l = lambda[4 * q + v];
    for (int d = 0; d < 3; ++d) x[d] += l * mesh.d_coords[3 * id + d];
  }
  for (int d = 0; d < 3; ++d) xyz[3 * i + d] = x[d];
}

__global__ void k_face_qp(hdg_mesh mesh, const double* __restrict__ xi, int nqd2, const int* __restrict__ list,
                          int n, double* __restrict__ xyz) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)n * nqd2) return;
  const int e = (int)(i / nqd2), r = (int)(i % nqd2);
  const int f = list[e];
  double x[3] = {0, 0, 0};
  if (f >= 0 && f < mesh.nfc) {
    for (int v = 0; v < 3; ++v) {
      const int id = mesh.d_faces[3 * f + v];
      const double l = xi[3 * r + v];
      for (int d = 0; d < 3; ++d) x[d] += l * mesh.d_coords[3 * id + d];
    }
  }
  for (int d = 0; d < 3; ++d) xyz[3 * i + d] = x[d];
}

template <int D2, int NQD2>
__global__ void k_uhat_init(hdg_mesh mesh, Tables tb, const double* __restrict__ uD, double* __restrict__ uhat) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < (size_t)mesh.nfc * D2) uhat[i] = 0.0;
  (void)tb;
  (void)uD;
}

template <int D2, int NQD2>
__global__ void k_dirichlet(hdg_mesh mesh, Tables tb, const double* __restrict__ uD, double* __restrict__ uhat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mesh.ndir * D2) return;
  const int r = i / D2, c = i % D2;
  double s = 0;
  for (int p = 0; p < NQD2; ++p) s += tb.tri_w[p] * tb.D[p * D2 + c] * uD[(size_t)r * NQD2 + p];
  uhat[(size_t)mesh.d_dirfaces[r] * D2 + c] = s;
}

template <int D2, int NQD2>
__global__ void k_neumann(hdg_mesh mesh, Tables tb, const double* __restrict__ gN, double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mesh.nneu * D2) return;
  const int r = i / D2, c = i % D2;
  const int f = mesh.d_neufaces[r];
  const int* g = mesh.d_faces + 3 * f;
  double u[3], w[3];
  for (int d = 0; d < 3; ++d) {
    u[d] = mesh.d_coords[3 * g[1] + d] - mesh.d_coords[3 * g[0] + d];
    w[d] = mesh.d_coords[3 * g[2] + d] - mesh.d_coords[3 * g[0] + d];
  }
  const double n0 = 0.5 * (u[1] * w[2] - u[2] * w[1]), n1 = 0.5 * (u[2] * w[0] - u[0] * w[2]),
               n2 = 0.5 * (u[0] * w[1] - u[1] * w[0]);
  double s = 0;
  for (int p = 0; p < NQD2; ++p) {
    const double* gp = gN + ((size_t)r * NQD2 + p) * 3;
    s += tb.tri_w[p] * tb.D[p * D2 + c] * (n0 * gp[0] + n1 * gp[1] + n2 * gp[2]);
  }
  F[(size_t)f * D2 + c] += s;
}

// Dirichlet elimination (eq 6.5 with the Dirichlet traces known): a Dirichlet row becomes
// the identity with right-hand side uhat; every other row subtracts H_fg uhat_g for its
// Dirichlet columns g (ascending block order) and clears those blocks.  Only rows that
// hold a Dirichlet column need work, and every such row is reached from the Dirichlet
// faces: thread (Dirichlet face g, local face l of g's element, row component c) takes row
// f = face l of that element, a Dirichlet row itself when l is g's own slot.  A row with
// several Dirichlet columns is processed by the thread of the smallest of them only, so
// each row is updated once and in the same order as a scan over all rows.
template <int D2>
__global__ void k_mask(hdg_mesh mesh, double* __restrict__ H, double* __restrict__ b, const double* __restrict__ uhat) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= mesh.ndir * 4 * D2) return;
  const int c = (int)(t % D2), l = (int)(t / D2 % 4), g = mesh.d_dirfaces[t / (4 * D2)];
  const int em = mesh.d_face_elem[2 * g];  // 4 E + m: the one element of a boundary face
  const int f = mesh.d_facebyele[(em & ~3) + l];
  const bool own = f == g;
  if (!own && mesh.d_ftype[f] == 1) return;  // another Dirichlet row: its own thread clears it
  const int p0 = mesh.d_row_ptr[f], p1 = mesh.d_row_ptr[f + 1];
  const size_t i = (size_t)f * D2 + c;
  if (own) {
    for (int p = p0; p < p1; ++p) {
      double* blk = H + ((size_t)p * D2 + c) * D2;
      const bool dg = mesh.d_col_idx[p] == f;
      for (int j = 0; j < D2; ++j) blk[j] = (dg && j == c) ? 1.0 : 0.0;
    }
    b[i] = uhat[i];
    return;
  }
  int gmin = INT_MAX;
  for (int p = p0; p < p1; ++p) {
    const int col = mesh.d_col_idx[p];
    if (mesh.d_ftype[col] == 1) gmin = min(gmin, col);
  }
  if (gmin != g) return;  // the row belongs to the thread of its smallest Dirichlet column
  double s = b[i];
  for (int p = p0; p < p1; ++p) {
    const int col = mesh.d_col_idx[p];
    if (mesh.d_ftype[col] != 1) continue;
    double* blk = H + ((size_t)p * D2 + c) * D2;
    for (int j = 0; j < D2; ++j) {
      s -= blk[j] * uhat[(size_t)col * D2 + j];
      blk[j] = 0.0;
    }
  }
  b[i] = s;
}

template <int K>
hdg_status run_boundary(const hdg_disc* disc, const hdg_mesh* mesh, const double* uD, const double* gN, double* H,
                        double* F, double* uhat, hipStream_t s) {
  using Dm = Dims<K>;
  constexpr int T = 256;
  const size_t nu = (size_t)mesh->nfc * Dm::D2;
  k_uhat_init<Dm::D2, Dm::NQD2><<<(unsigned)((nu + T - 1) / T), T, 0, s>>>(*mesh, disc->dev, uD, uhat);
  if (mesh->ndir)
    k_dirichlet<Dm::D2, Dm::NQD2><<<(unsigned)((mesh->ndir * Dm::D2 + T - 1) / T), T, 0, s>>>(*mesh, disc->dev, uD, uhat);
  if (mesh->nneu)
    k_neumann<Dm::D2, Dm::NQD2><<<(unsigned)((mesh->nneu * Dm::D2 + T - 1) / T), T, 0, s>>>(*mesh, disc->dev, gN, F);
  if (mesh->ndir) {
    const size_t nm = (size_t)mesh->ndir * 4 * Dm::D2;
    k_mask<Dm::D2><<<(unsigned)((nm + T - 1) / T), T, 0, s>>>(*mesh, H, F, uhat);
  }
  HDG_CHECK_LAUNCH("hdg_boundary");
  return HDG_OK;
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, double* d_xyz, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_qp_coords");
  if (st) return st;
  if (!d_xyz) return set_error(HDG_ERR_INVALID_ARG, "hdg_qp_coords: NULL output");
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)mesh->nelt * disc->host.nqd;
  const unsigned grid = (unsigned)((n + 255) / 256);
  switch (disc->host.k) {
    case 0: k_qp_coords<Dims<0>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 1: k_qp_coords<Dims<1>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 2: k_qp_coords<Dims<2>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 3: k_qp_coords<Dims<3>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 4: k_qp_coords<Dims<4>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 5: k_qp_coords<Dims<5>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    case 6: k_qp_coords<Dims<6>::NQD><<<grid, 256, 0, s>>>(*mesh, disc->d_tables + disc->host.off.lambda, d_xyz); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_qp_coords: unsupported degree");
  }
  HDG_CHECK_LAUNCH("hdg_qp_coords");
  return HDG_OK;
}

extern "C" hdg_status hdg_face_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, const int32_t* d_faces_list,
                                         int64_t n, double* d_xyz, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_face_qp_coords");
  if (st) return st;
  if (n < 0 || (n && (!d_faces_list || !d_xyz)))
    return set_error(HDG_ERR_INVALID_ARG, "hdg_face_qp_coords: bad arguments");
  if (n == 0) return HDG_OK;
  const size_t tot = (size_t)n * disc->host.nqd2;
  k_face_qp<<<(unsigned)((tot + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      *mesh, disc->d_tables + disc->host.off.xi, disc->host.nqd2, d_faces_list, (int)n, d_xyz);
  HDG_CHECK_LAUNCH("hdg_face_qp_coords");
  return HDG_OK;
}

extern "C" hdg_status hdg_boundary(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_uD,
                                   const double* d_gN, double* d_H, double* d_F, double* d_uhat, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_boundary");
  if (st) return st;
  if (!d_H || !d_F || !d_uhat || (mesh->ndir && (!d_uD || !mesh->d_dirfaces)) ||
      (mesh->nneu && (!d_gN || !mesh->d_neufaces)) || !mesh->d_row_ptr || !mesh->d_col_idx || !mesh->d_ftype)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_boundary: NULL array");
  hipStream_t s = (hipStream_t)stream;
  switch (disc->host.k) {
    case 0: return run_boundary<0>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 1: return run_boundary<1>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 2: return run_boundary<2>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 3: return run_boundary<3>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 4: return run_boundary<4>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 5: return run_boundary<5>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
    case 6: return run_boundary<6>(disc, mesh, d_uD, d_gN, d_H, d_F, d_uhat, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_boundary: unsupported degree");
}
