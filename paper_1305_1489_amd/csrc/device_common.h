// Device-side helpers shared by the element kernels.
#pragma once

#include "hdg_internal.h"

namespace hdg {

template <int K>
struct Dims {
  static constexpr int D3 = dim3(K);
  static constexpr int D2 = dim2(K);
  static constexpr int M = 4 * D2;
  static constexpr int NQ = K + 2;
  static constexpr int NQD = NQ * NQ * NQ;
  static constexpr int NQD2 = NQ * NQ;
  static constexpr int D3P = dim3(K + 1);
};

// Geometry of one element (eq 2.0, eq 3.8, Section 2): a = det(B) B^{-T} (the cofactor
// matrix, a[s][h] = a_{s h}), |K|, outward normals n_l with |n_l| = |e_l|, T_l = tau_l |e_l|,
// and mu_l = perm(K, l) - 1.
// A pointer read from device memory (a batch work item) is a generic pointer, and the
// compiler then emits flat memory instructions for it; a flat access also counts against
// the LDS wait counter, so every later LDS wait waits for it to reach memory.  as_global
// states that the pointer addresses global memory (it always does here), after which its
// accesses are compiled as global ones.
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}
__device__ __forceinline__ hdg_mesh as_global(const hdg_mesh& m) {
  hdg_mesh g = m;
  g.d_coords = as_global(g.d_coords);
  g.d_elements = as_global(g.d_elements);
  g.d_dirichlet = as_global(g.d_dirichlet);
  g.d_neumann = as_global(g.d_neumann);
  g.d_faces = as_global(g.d_faces);
  g.d_ftype = as_global(g.d_ftype);
  g.d_dirfaces = as_global(g.d_dirfaces);
  g.d_neufaces = as_global(g.d_neufaces);
  g.d_facebyele = as_global(g.d_facebyele);
  g.d_perm = as_global(g.d_perm);
  g.d_volume = as_global(g.d_volume);
  g.d_area = as_global(g.d_area);
  g.d_normals = as_global(g.d_normals);
  g.d_face_elem = as_global(g.d_face_elem);
  g.d_row_ptr = as_global(g.d_row_ptr);
  g.d_col_idx = as_global(g.d_col_idx);
  g.d_diag = as_global(g.d_diag);
  g.d_slot = as_global(g.d_slot);
  return g;
}

struct ElemGeom {
  double v0[3];
  double a[3][3];
  double det, vol;
  double n[4][3];
  double T[4];
  int mu[4];
};

__device__ inline void load_geometry(int K, const hdg_mesh& mesh, const double* __restrict__ tau, ElemGeom& g) {
  // no FMA contraction: every kernel, whichever way it is compiled, gets the same bits
#pragma clang fp contract(off)
  const int* el = mesh.d_elements + 4 * K;
  double p[4][3];
  for (int i = 0; i < 4; ++i) {
    int v = el[i];
    for (int d = 0; d < 3; ++d) p[i][d] = mesh.d_coords[3 * v + d];
  }
  double e1[3], e2[3], e3[3];
  for (int d = 0; d < 3; ++d) {
    g.v0[d] = p[0][d];
    e1[d] = p[1][d] - p[0][d];
    e2[d] = p[2][d] - p[0][d];
    e3[d] = p[3][d] - p[0][d];
  }
  // columns of a: e2 x e3, e3 x e1, e1 x e2
  double c0[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
  double c1[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
  double c2[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  for (int s = 0; s < 3; ++s) {
    g.a[s][0] = c0[s];
    g.a[s][1] = c1[s];
    g.a[s][2] = c2[s];
  }
  g.det = c2[0] * e3[0] + c2[1] * e3[1] + c2[2] * e3[2];
  g.vol = g.det / 6.0;
  const double* nn = mesh.d_normals + 12 * K;
  for (int l = 0; l < 4; ++l) {
    double s2 = 0;
    for (int d = 0; d < 3; ++d) {
      g.n[l][d] = nn[3 * l + d];
      s2 += g.n[l][d] * g.n[l][d];
    }
    g.T[l] = tau ? tau[4 * K + l] * sqrt(s2) : 0.0;  // no tau: the mixed (BDM) element
    g.mu[l] = mesh.d_perm[4 * K + l] - 1;
  }
}

// Cholesky factorisation in place of an n x n SPD matrix in LDS (row-major, leading
// dimension ld); the lower triangle receives L.  All threads of the block take part.
template <int N>
__device__ inline void lds_cholesky(double* A, int ld) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < N; ++j) {
    if (t == 0) {
      double s = A[j * ld + j];
      for (int k = 0; k < j; ++k) s -= A[j * ld + k] * A[j * ld + k];
      A[j * ld + j] = sqrt(s);
    }
    __syncthreads();
    const double inv = 1.0 / A[j * ld + j];
    for (int i = j + 1 + t; i < N; i += nt) {
      double s = A[i * ld + j];
      for (int k = 0; k < j; ++k) s -= A[i * ld + k] * A[j * ld + k];
      A[i * ld + j] = s * inv;
    }
    __syncthreads();
  }
}

// X <- L^{-1} X for NC columns of an N-row matrix X (row-major, leading dimension ldx),
// L lower triangular (ld ldl).  One thread per column.
template <int N>
__device__ inline void lds_forward_cols(const double* L, int ldl, double* X, int ldx, int ncols) {
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    for (int r = 0; r < N; ++r) {
      double s = X[r * ldx + c];
      for (int k = 0; k < r; ++k) s -= L[r * ldl + k] * X[k * ldx + c];
      X[r * ldx + c] = s / L[r * ldl + r];
    }
  }
}

// X <- L^{-T} X (back substitution with the transpose), one thread per column.
template <int N>
__device__ inline void lds_backward_cols(const double* L, int ldl, double* X, int ldx, int ncols) {
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    for (int r = N - 1; r >= 0; --r) {
      double s = X[r * ldx + c];
      for (int k = r + 1; k < N; ++k) s -= L[k * ldl + r] * X[k * ldx + c];
      X[r * ldx + c] = s / L[r * ldl + r];
    }
  }
}

// ---- batched (several meshes per launch) persistent kernels

// Index of the mesh owning work unit u: the last item whose unit_begin <= u.  The unit is
// uniform over the workgroup, so the search runs on the scalar unit.
__device__ __forceinline__ int batch_find(const BatchItem* __restrict__ items, int n, int u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Workgroups are dealt round-robin to the eight XCDs (workgroup b runs on XCD b mod 8).
// With remapping, the workgroups of one XCD take consecutive unit numbers, so that
// neighbouring elements (which share vertices, faces and rows of H) meet in one L2.
__device__ __forceinline__ int batch_block(int xcd_remap) {
  const int b = blockIdx.x, nb = gridDim.x;
  if (!xcd_remap || (nb & 7)) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Geometry record of one element, the layout shared by the tile condensation (which
// precomputes it or keeps it in LDS, and stores it with the element's factors) and the
// tile reconstruction (which reads it back).
// G_DU holds the number of degree-k modes removed from the scalar space (0 for HDG, d2 for
// the hybridized BDM element, whose u lives in P_{k-1}); the reconstruction reads it.
enum { G_A = 0, G_DET = 9, G_VOL = 10, G_N = 11, G_T = 23, G_NN = 27, G_MU = 43, G_DU = 47, G_REC = kGeoRecord };
static_assert(G_DU < G_REC, "geometry record layout");

// The geometry record of element E (E < 0: a reference element with no data), laid out as
// above, perm - 1 and the removed-mode count stored as small integers in doubles; tau may be
// NULL (T_l = 0).  No FMA contraction here or in
// load_geometry, so that the records precomputed by k_geo_records and the ones computed
// inline by the other forms of the condensation are the same bits.
__device__ inline void tile_geo_record(int E, const hdg_mesh& mesh, const double* __restrict__ tau, double* rec,
                                       int du_removed = 0) {
#pragma clang fp contract(off)
  ElemGeom g;
  if (E >= 0) {
    load_geometry(E, mesh, tau, g);
  } else {
    g = ElemGeom{};
    g.vol = 1.0;
    g.det = 6.0;
  }
  for (int i = 0; i < 9; ++i) rec[G_A + i] = g.a[i / 3][i % 3];
  rec[G_DET] = g.det;
  rec[G_VOL] = g.vol;
  for (int i = 0; i < 12; ++i) rec[G_N + i] = g.n[i / 3][i % 3];
  for (int l = 0; l < 4; ++l) {
    rec[G_T + l] = g.T[l];
    rec[G_MU + l] = (double)g.mu[l];
    for (int m = 0; m < 4; ++m)
      rec[G_NN + 4 * l + m] = g.n[l][0] * g.n[m][0] + g.n[l][1] * g.n[m][1] + g.n[l][2] * g.n[m][2];
  }
  for (int i = G_MU + 4; i < G_REC; ++i) rec[i] = 0.0;
  rec[G_DU] = (double)du_removed;
}

}  // namespace hdg
