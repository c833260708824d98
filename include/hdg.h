/*
 * hdg.h -- C ABI of libhdg: the element-local hot path of the hybridizable
 * discontinuous Galerkin (HDG) method for variable-coefficient reaction-diffusion
 *
 *     kappa^{-1} q + grad u = 0,   div q + c u = f   in Omega,
 *     u = u_D on Gamma_D,          -q . nu = g_N . nu on Gamma_N          (eq 1.1)
 *
 * on conforming tetrahedral meshes with polynomial degree k (Fu, Gatica, Sayas,
 * "Matlab tools for HDG in three dimensions").  The hybrid unknown uhat lives on
 * faces; q and u are eliminated element by element (Section 5) and recovered after
 * the global solve (Section 6).
 *
 * Conventions shared by every call
 *   - Every call returns hdg_status (HDG_OK = 0).  hdg_last_error() returns a
 *     thread-local message for the last failing call.  No C++ exception crosses
 *     the ABI.  Arguments are validated on the host before any launch, so a call
 *     that fails validation writes nothing.
 *   - Pointers named d_* are device pointers (HIP device memory of the current
 *     device), owned by the caller, who keeps them alive for as long as any handle
 *     refers to them.  Host pointers are named h_*.  Compute calls are
 *     asynchronous on the caller's stream and allocate no device memory; they are
 *     safe to capture into a HIP graph unless stated otherwise.  Scratch memory is
 *     passed in as a workspace whose size the matching *_workspace_size call gives.
 *   - Indices are 0-based int32 (the paper's are 1-based).  Dense per-element
 *     arrays are element-major ("[Nelt][...]", the element's entries contiguous).
 *   - A device fault raised by an earlier asynchronous launch surfaces at the next
 *     call that synchronises, as HDG_ERR_DEVICE.
 *   - Handles are not thread-safe; use one per thread.
 *
 * Dimensions: d3 = C(k+3,3) (dim P_k(K)), d2 = C(k+2,2) (dim P_k(e)), m = 4 d2,
 * d3p = C(k+4,3) (dim P_{k+1}(K)); the volume rule has nqd = n^3 points and the
 * face rule nqd2 = n^2 points, n = k+2 unless chosen otherwise.
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hdg_status;
enum {
  HDG_OK = 0,
  HDG_ERR_INVALID_ARG = 1,
  HDG_ERR_UNSUPPORTED_DEGREE = 2,
  HDG_ERR_MESH_ORIENTATION = 3,   /* element with det B_K <= 0, or inward boundary triangle */
  HDG_ERR_MESH_NONCONFORMING = 4, /* a face shared by more than two elements               */
  HDG_ERR_BOUNDARY_UNLISTED = 5,  /* a boundary face in neither list                        */
  HDG_ERR_BOUNDARY_INVALID = 6,   /* a listed triangle that is not a boundary face, or listed twice */
  HDG_ERR_TAU_ZERO = 7,           /* tau vanishes on all four faces of an element, or tau < 0 */
  HDG_ERR_WORKSPACE = 8,          /* workspace pointer null or too small                   */
  HDG_ERR_DEVICE = 9,             /* a HIP runtime error                                   */
  HDG_ERR_NOT_CONVERGED = 10,     /* iterative solve stopped before the tolerance          */
  HDG_ERR_SINGULAR = 11           /* no Dirichlet face and c == 0: constants in the kernel  */
};

/* Thread-local message describing the last failing call (never NULL). */
const char* hdg_last_error(void);

/* Largest supported polynomial degree (6).  Degrees 0..6 have the whole path (condensation,
 * boundary data, PCG, reconstruction, postprocess); the batched, FP32-refined, learned,
 * export and non-symmetric forms stop at the degrees their entries state. */
int hdg_max_degree(void);

/* Measurement hook (no effect on results): while set, every launch by this thread of the
 * library kernel named `kernel` ("k_condense_tile", "k_condense", "k_geo_records",
 * "k_diag_sum", "k_recover_tile", "k_recover", "k_pp_rhs", "k_pp_solve", "k_face_moments",
 * "k_hdg_projection") is bracketed by
 * hipEventRecord(ev_start) and hipEventRecord(ev_stop) on the stream of the call, so that
 * one kernel of a multi-kernel call can be timed with the caller's events (hipEvent_t,
 * created and owned by the caller, timing enabled).  kernel = NULL switches it off.
 * Errors: HDG_ERR_INVALID_ARG (a NULL event with a non-NULL name). */
hdg_status hdg_set_kernel_timer(const char* kernel, void* ev_start, void* ev_stop);

/* ------------------------------------------------------------------------------
 * Mesh (Section 2, "Data structure").
 *
 * Basic form (input of hdg_mesh_expand):
 *   d_coords    double [nver][3]        vertex coordinates
 *   d_elements  int32  [nelt][4]        vertex numbers, positively oriented
 *   d_dirichlet int32  [ndir][3]        Dirichlet triangles, outward orientation
 *   d_neumann   int32  [nneu][3]        Neumann triangles, outward orientation
 * Expanded form (outputs of hdg_mesh_expand, sized by hdg_mesh_sizes):
 *   d_faces     int32  [nfc][3]  vertex numbers; the order fixes the face's own
 *                                parametrisation phi_e (Section 2).  Faces are
 *                                numbered by ascending sorted vertex triple; a
 *                                boundary face keeps the order of its row in the
 *                                Dirichlet/Neumann list, an interior face the local
 *                                order (eq 2.1) of its lower-numbered element.
 *   d_ftype     int32  [nfc]     0 interior, 1 Dirichlet, 2 Neumann
 *   d_dirfaces  int32  [ndir]    face number of each Dirichlet row
 *   d_neufaces  int32  [nneu]    face number of each Neumann row
 *   d_facebyele int32  [nelt][4] faces of each element in the order of eq 2.1
 *   d_perm      int32  [nelt][4] perm(K, l) in 1..6 (eq 2.2-2.3)
 *   d_volume    double [nelt]    |K|
 *   d_area      double [nfc]     |e|
 *   d_normals   double [nelt][4][3] outward normals with |n_l| = |e_l|
 *   d_face_elem int32  [nfc][2]  4K+l of the (one or two) elements holding the face,
 *                                ascending; -1 in the second slot on the boundary
 *   global trace system H (eq 6.5) in block-sparse-row form with d2 x d2 blocks:
 *   d_row_ptr   int32  [nfc+1]   block-row pointers
 *   d_col_idx   int32  [nnzb]    block columns, ascending within a row
 *   d_diag      int32  [nfc]     block index of the diagonal block of each row
 *   d_slot      int32  [nelt][16] block index of (facebyele[K][l], facebyele[K][m])
 *                                at entry 4l+m: where the (l,m) block of C^K goes
 * ------------------------------------------------------------------------------ */
typedef struct {
  int64_t nver, nelt, ndir, nneu;
  int64_t nfc;   /* = (4 nelt + ndir + nneu) / 2 for a valid mesh  */
  int64_t nnzb;  /* = nfc + 12 nelt                                 */
  const double* d_coords;
  const int32_t* d_elements;
  const int32_t* d_dirichlet;
  const int32_t* d_neumann;
  int32_t* d_faces;
  int32_t* d_ftype;
  int32_t* d_dirfaces;
  int32_t* d_neufaces;
  int32_t* d_facebyele;
  int32_t* d_perm;
  double* d_volume;
  double* d_area;
  double* d_normals;
  int32_t* d_face_elem;
  int32_t* d_row_ptr;
  int32_t* d_col_idx;
  int32_t* d_diag;
  int32_t* d_slot;
} hdg_mesh;

/* Fills nfc and nnzb of *mesh from nver/nelt/ndir/nneu (which the caller sets) and
 * returns the workspace size of hdg_mesh_expand in *ws_bytes.
 * Errors: HDG_ERR_INVALID_ARG (negative sizes, odd 4 nelt + ndir + nneu, or more
 * than 2^21 vertices). */
hdg_status hdg_mesh_sizes(hdg_mesh* mesh, size_t* ws_bytes);

/* Expanded mesh from the basic one (Section 2): face list by a stable radix sort of
 * sorted-vertex-triple keys and a segmented unique, facebyele, perm, volumes,
 * areas, outward normals, and the block pattern of H with the per-element slot map.
 * All integer outputs are deterministic.  Synchronises the stream once at the end
 * to read the validation flag (setup call, not graph-capturable).
 * Errors: HDG_ERR_MESH_ORIENTATION, HDG_ERR_MESH_NONCONFORMING,
 * HDG_ERR_BOUNDARY_UNLISTED, HDG_ERR_BOUNDARY_INVALID, HDG_ERR_WORKSPACE,
 * HDG_ERR_INVALID_ARG, HDG_ERR_DEVICE.  On error the outputs are unspecified. */
hdg_status hdg_mesh_expand(hdg_mesh* mesh, void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------
 * Discretisation: reference-element tables for degree k (Sections 3-4).
 * Stroud conical-product Gauss-Jacobi rules with nq points per collapsed direction
 * (nq = 0 selects k + 2, exact to degree 2k + 3), orthonormal hierarchical Dubiner
 * bases, and the reference matrices C^x,y,z (eq 3.7), PP_l (eq 4.5), DP_{mu,l}
 * (eq 4.10), and the stiffness tables of P_{k+1} used by the postprocess.
 * Tables are built on the host in long double and uploaded once to a device
 * buffer that the handle owns (setup-time allocation; freed by destroy).
 * ------------------------------------------------------------------------------ */
typedef struct hdg_disc hdg_disc;

typedef struct {
  int k, nq, d3, d2, m, d3p, nqd, nqd2;
  int factor_len;   /* doubles per element in the factor store (see hdg_assemble_condense) */
} hdg_disc_info;

/* Errors: HDG_ERR_UNSUPPORTED_DEGREE (k < 0 or k > hdg_max_degree()),
 * HDG_ERR_INVALID_ARG (nq < k+1 or nq > 8), HDG_ERR_DEVICE. */
hdg_status hdg_disc_create(int k, int nq, hdg_disc** out);
hdg_status hdg_disc_destroy(hdg_disc* disc);
hdg_status hdg_disc_get_info(const hdg_disc* disc, hdg_disc_info* info);
/* Copies host copies of the tables (for tests): name is one of "vol_pts" [nqd][3],
 * "vol_w" [nqd], "tri_pts" [nqd2][2], "tri_w" [nqd2], "P" [nqd][d3], "Pgrad"
 * [3][nqd][d3], "D" [nqd2][d2], "Pface" [4][nqd2][d3], "Chat" [3][d3][d3],
 * "PP" [4][d3][d3], "DP" [6][4][d2][d3], "P1grad" [3][nqd][d3p], "Shat"
 * [6][d3p][d3p] (xx, yy, zz, xy+yx, xz+zx, yz+zy), "DPtopinv" [6][4][d2][d2] (the inverse of
 * the last d2 columns of each DP_{mu,l}, used by the HDG projection), "Dmu" [6][nqd2][d2] (the
 * face basis at F_mu(qhat_r), eq 2.2), and the zero-padded layouts of the
 * postprocess kernel: "P1grad_pad" [3][nqp][d3pp4] and "Shat_tiles" [6][ts(ts+1)/2][4][4]
 * (upper 4x4 tiles (I, N), I <= N, row by row), where nqp and d3pp4 are nqd and d3p
 * rounded up to multiples of 4 and ts = d3pp4 / 4.  *count receives the number of
 * doubles; pass h_out = NULL to query it. */
hdg_status hdg_disc_table(const hdg_disc* disc, const char* name, double* h_out, int64_t* count);

/* Host-only variant of hdg_disc_table that needs no device: builds the tables of
 * degree k with nq points per direction (0: k+2) on the host and copies the named one.
 * Errors: HDG_ERR_UNSUPPORTED_DEGREE, HDG_ERR_INVALID_ARG. */
hdg_status hdg_reference_table(int k, int nq, const char* name, double* h_out, int64_t* count);

/* Physical volume quadrature points x_q = F_K(p_q) (eq 3.2, 3.4):
 * d_xyz double [nelt][nqd][3].  The caller evaluates kappa, c and f there. */
hdg_status hdg_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, double* d_xyz, void* stream);

/* Face quadrature points y_r = phi_e(qhat_r) in each listed face's own
 * parametrisation (Section 4, eq 6.2): d_faces_list int32 [n] face numbers,
 * d_xyz double [n][nqd2][3]. */
hdg_status hdg_face_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, const int32_t* d_faces_list,
                              int64_t n, double* d_xyz, void* stream);

/* ------------------------------------------------------------------------------
 * Assembly + static condensation + scatter (Sections 3-6, eq 5.1-5.6, eq 6.5).
 *   d_kappa, d_c, d_f  double [nelt][nqd]  kappa > 0, c >= 0 and f at the points of
 *                                          hdg_qp_coords
 *   d_tau              double [nelt][4]    tau_K on the faces of K in facebyele order
 *                                          (>= 0, not all zero on an element)
 * Outputs:
 *   d_H       double [nnzb][d2][d2]  the block-sparse trace matrix of eq 6.5
 *                                    (row-major blocks); exactly symmetric
 *   d_F       double [nfc][d2]       the assembled Cf (eq 6.5's F)
 *   d_factors double [nelt][factor_len]  per-element factors kept for hdg_recover:
 *                                    the factors of M_{1/kappa} and of the u-Schur
 *                                    complement, f^K, and (degrees 1..3) the element's
 *                                    geometry record, so that hdg_recover does not
 *                                    recompute it; opaque to the caller
 * Every block of H and every entry of F is written; off-diagonal blocks have one
 * contributing element, diagonal blocks and F entries at most two, summed in an
 * order-independent way, so results are bitwise reproducible.
 * Degrees 5 and 6 keep each element's solved blocks (the columns L^{-1} [C^T | DP^T] and
 * Ls^{-1} [B | f], 147 KB per element at k = 5 and 313 KB at k = 6) in a caller workspace,
 * so this entry, which takes none, returns HDG_ERR_WORKSPACE for them: use
 * hdg_assemble_condense_ws (or hdg_assemble_condense_noalloc).
 * Errors: HDG_ERR_INVALID_ARG; HDG_ERR_SINGULAR when the mesh has no Dirichlet face and
 * c == 0 at every volume point (Section 1: constants then solve the homogeneous system).
 * That check runs only for meshes without Dirichlet faces; it reads one flag back and so
 * synchronises the stream (such a call is not graph-capturable).  Tau validity is the
 * caller's contract (not checked on the device; hdg_check_tau checks it). */
hdg_status hdg_assemble_condense(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                 const double* d_c, const double* d_f, const double* d_tau, double* d_H,
                                 double* d_F, double* d_factors, void* stream);

/* Host check of tau (copies d_tau to the host; synchronises). HDG_ERR_TAU_ZERO. */
hdg_status hdg_check_tau(const hdg_mesh* mesh, const double* d_tau, void* stream);

/* Debug / parity export: C^K (m x m, row-major) and Cf^K for the listed elements,
 * computed by the same device code as hdg_assemble_condense.  Degrees 0..4
 * (HDG_ERR_UNSUPPORTED_DEGREE above).
 *   d_elems int32 [n], d_C double [n][m][m], d_Cf double [n][m]. */
hdg_status hdg_export_local(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa, const double* d_c,
                            const double* d_f, const double* d_tau, const int32_t* d_elems, int64_t n,
                            double* d_C, double* d_Cf, void* stream);

/* ------------------------------------------------------------------------------
 * Boundary conditions (eq 6.1-6.4 and the elimination at the end of Section 6).
 *   d_uD   double [ndir][nqd2]     u_D at the face points of the Dirichlet faces
 *                                  (hdg_face_qp_coords of d_dirfaces)
 *   d_gN   double [nneu][nqd2][3]  the Neumann vector field g_N at the points of the
 *                                  Neumann faces (only g_N . n_e is used)
 * In place on the output of hdg_assemble_condense:
 *   d_F    becomes the right-hand side b of the reduced system: F + G_N on free
 *          faces minus H_ID uD, uD on Dirichlet faces
 *   d_H    Dirichlet rows/columns are replaced by identity/zero blocks, so that the
 *          system stays symmetric positive definite
 *   d_uhat double [nfc][d2] is set to uD on Dirichlet faces and 0 elsewhere
 * Errors: HDG_ERR_INVALID_ARG. */
hdg_status hdg_boundary(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_uD, const double* d_gN,
                        double* d_H, double* d_F, double* d_uhat, void* stream);

/* ------------------------------------------------------------------------------
 * Global solve of the trace system H uhat = b (eq 6.5; the paper leaves the solver
 * open): preconditioned conjugate gradients with a block-Jacobi preconditioner
 * (Cholesky of the d2 x d2 diagonal blocks), FP64, deterministic reductions,
 * stopping when the recomputed FP64 residual satisfies ||b - H x|| <= rtol ||b||.
 * d_uhat is the initial guess on entry (Dirichlet values included) and the
 * solution on exit.  The host reads one scalar every check_every iterations.
 * ------------------------------------------------------------------------------ */
typedef struct {
  double rtol;        /* relative residual target, e.g. 1e-10 */
  int max_iter;
  int check_every;    /* iterations between host convergence checks (>= 1) */
  int precision;      /* 0: FP64 throughout; 1: FP32 matrix and preconditioner inside
                         an FP64 iterative-refinement loop */
  int precond;        /* 0: block-Jacobi; 1: learned factor (needs the three arrays below;
                         degrees 0..4, else HDG_ERR_UNSUPPORTED_DEGREE) */
  const float* d_pre_N;      /* [nnzb][d2][d2] N of the learned factor, lower blocks and their
                                transposes at the mirrored positions (hdg_gnn_forward) */
  const float* d_pre_Linv;   /* [nfc][d2][d2]  hdg_gnn_graph.Linv */
  const float* d_pre_B;      /* [nfc][d2 (d2 + 1) / 2] block scaling of the learned factor
                                (hdg_gnn_forward), or NULL for B = I */
} hdg_solve_opts;

typedef struct {
  int iterations;     /* total inner iterations (both attempts when fell_back) */
  int outer;          /* refinement sweeps (precision 1) */
  double rel_residual;/* true relative residual ||b - H x|| / ||b|| in FP64 */
  int fell_back;      /* 1: the learned-preconditioner run did not converge and block-Jacobi
                         PCG finished the solve */
} hdg_solve_info;

hdg_status hdg_solve_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, int precision, size_t* ws_bytes);
hdg_status hdg_solve(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, const double* d_b,
                     double* d_uhat, const hdg_solve_opts* opts, hdg_solve_info* info, void* d_ws,
                     size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------
 * Reconstruction and postprocess (Section 6 "Reconstruction", eq 5.3, eq 9.11).
 *   d_factors  from hdg_assemble_condense (same disc, mesh, coefficients, tau)
 *   d_kappa    double [nelt][nqd] (for the postprocess right-hand side)
 *   d_tau      double [nelt][4]
 *   d_uhat     double [nfc][d2]
 * Outputs: d_q double [nelt][3][d3], d_u double [nelt][d3],
 *          d_ustar double [nelt][d3p] (may be NULL to skip the postprocess).
 * ------------------------------------------------------------------------------ */
hdg_status hdg_recover(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa, const double* d_tau,
                       const double* d_factors, const double* d_uhat, double* d_q, double* d_u,
                       double* d_ustar, void* stream);

/* ------------------------------------------------------------------------------
 * Local postprocess alone (eq 9.11): u* in P_{k+1}(K) with grad u* = -kappa^{-1} q_h
 * in the least-squares sense on K (the stiffness system tested against the gradients of
 * P_{k+1}) and the mean of u* equal to that of u_h.  hdg_recover with a non-NULL d_ustar
 * runs it after the reconstruction; this entry runs it on given fields.
 *   d_kappa  double [nelt][nqd]     d_tau double [nelt][4] (geometry set-up only)
 *   d_q      double [nelt][3][d3]   d_u   double [nelt][d3]   (layouts of hdg_recover)
 *   d_factors  the factor store of hdg_assemble_condense(_ws) for the same mesh and tau,
 *            or NULL: for degrees 1..3 the element geometry is then read from it instead
 *            of recomputed (same values); ignored for degrees 0, 4, 5 and 6
 * Output: d_ustar double [nelt][d3p].  Errors: HDG_ERR_INVALID_ARG (NULL array),
 * HDG_ERR_UNSUPPORTED_DEGREE, HDG_ERR_DEVICE.  Nothing is allocated.
 * ------------------------------------------------------------------------------ */
hdg_status hdg_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa, const double* d_tau,
                           const double* d_q, const double* d_u, const double* d_factors, double* d_ustar,
                           void* stream);

/* Same results as hdg_assemble_condense, bit for bit, without atomics.  Each element's
 * contributions to its diagonal face blocks and to F go to the caller's workspace (the
 * upper triangle of a d2 x d2 block and d2 entries per (element, face)), and a second
 * kernel sums the one or two contributions of each face in a fixed order.  A first kernel
 * writes each element's geometry (48 doubles) into the workspace as well, so that the
 * condensation loads it in one pass.  Workspace: hdg_condense_workspace_size bytes =
 * round_up(4 Nelt (d2 (d2 + 1) / 2 + d2) 8, 256) + 384 Nelt, device memory owned by the
 * caller, contents undefined on entry and exit (0 for degrees 0 and 4, which always use
 * the atomic scatter).  Degrees 5 and 6 scatter with the two-addend atomics as well and use
 * the workspace for the element blocks: one slice of d3 (3 d3 + 4 d2) + d3 (4 d2 + 1)
 * doubles per workgroup of the persistent grid (workgroups_per_cu of hdg_set_launch_config
 * times the compute units, at most Nelt): 37.7 MB at k = 5 and 80 MB at k = 6 on 256
 * compute units.  Errors: those of hdg_assemble_condense, HDG_ERR_WORKSPACE. */
hdg_status hdg_condense_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes);
hdg_status hdg_assemble_condense_ws(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                    const double* d_c, const double* d_f, const double* d_tau, double* d_H, double* d_F,
                                    double* d_factors, void* d_ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hdg_assemble_condense_ws with the
 * library's own workspace instead of the caller's.  That workspace is a static device array
 * of hdg_condense_noalloc_capacity() bytes (256 MiB), one per device the library runs on,
 * held until the process ends; the call itself allocates nothing.  The caller still passes
 * every input and output.  Same results as hdg_assemble_condense_ws, bit for bit.
 * Limit: hdg_condense_workspace_size(disc, mesh) must not exceed the capacity (k = 3: up to
 * about 108,000 elements; k = 2: 215,000; k = 1: 399,000; k = 0, 4 need none; k = 5, 6 any
 * mesh at one workgroup per compute unit), else
 * HDG_ERR_WORKSPACE before any launch.  Every call on a device shares that device's array
 * and leaves it in an undefined state: calls that overlap in time on one device (two
 * streams, two threads) race and must be serialised by the caller.  Errors: those of
 * hdg_assemble_condense_ws. */
hdg_status hdg_condense_noalloc_capacity(size_t* bytes);
hdg_status hdg_assemble_condense_noalloc(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                         const double* d_c, const double* d_f, const double* d_tau, double* d_H,
                                         double* d_F, double* d_factors, void* stream);

/* ------------------------------------------------------------------------------
 * Hybridized BDM element (Section 9, "BDM"), degrees 1..3: V_h = P_k(K)^3, W_h = P_{k-1}(K),
 * M_h as for HDG, tau = 0.  The local matrices are those of hdg_assemble_condense with tau = 0
 * and the last d2 rows and columns of A1 (the degree-k modes of u and of its test space), the
 * last d2 rows of A2 and Af and the last d2 columns of A3 deleted; C^K = A3 A1^{-1} A2 and
 * Cf^K = A3 A1^{-1} Af are scattered into H and F exactly as by hdg_assemble_condense_ws
 * (same workspace, same layouts).  The factor store records the element as BDM, so that
 * hdg_recover returns u in P_{k-1}(K) (its degree-k coefficients zero) and q in P_k(K)^3;
 * hdg_boundary and hdg_solve apply unchanged.  Errors: HDG_ERR_UNSUPPORTED_DEGREE (k = 0 or
 * 4), HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE, HDG_ERR_SINGULAR (as for hdg_assemble_condense).
 * ------------------------------------------------------------------------------ */
hdg_status hdg_assemble_condense_bdm(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                     const double* d_c, const double* d_f, double* d_H, double* d_F,
                                     double* d_factors, void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------
 * Local projections and the superconvergence diagnostics (Section 9, "Local L2
 * projections" and "HDG projection"; eq 9.12, 9.13, 10.2).  The caller evaluates the
 * fields at the library's quadrature points (hdg_qp_coords, hdg_face_qp_coords), as for the
 * coefficients.
 * ------------------------------------------------------------------------------ */
/* L2 projection onto M_h (eq 9.12) of ncomp fields on n faces: d_vals double
 * [n][nqd2][ncomp] holds the fields at the points of hdg_face_qp_coords of those faces (in
 * each face's own parametrisation); d_out double [n][ncomp][d2] receives the coefficients in
 * the orthonormal face basis (whose face mass matrix is the identity, so this is
 * (w . D)^T v, the formula of eq 6.3).  One thread per output, nothing allocated.
 * Errors: HDG_ERR_INVALID_ARG (NULL array, n < 0, ncomp outside 1..8). */
hdg_status hdg_project_trace(const hdg_disc* disc, const hdg_mesh* mesh, int64_t n, int ncomp, const double* d_vals,
                             double* d_out, void* stream);
/* HDG projection (eq 9.13): (Pi q, Pi u) in P_k(K)^3 x P_k(K) with the moments of q and u
 * against P_{k-1}(K) and, on every face, the moments of q.nu + tau u against P_k(e).
 *   d_tau      double [nelt][4]       as for the condensation (not zero on all four faces)
 *   d_qu_vol   double [nelt][nqd][4]  (q_x, q_y, q_z, u) at the points of hdg_qp_coords
 *                                     (32-byte aligned, as every hipMalloc'd buffer is)
 *   d_qu_face  double [nfc][nqd2][4]  the same at the points of hdg_face_qp_coords of faces
 *                                     0..nfc-1
 *   d_Pq       double [nelt][3][d3], d_Pu double [nelt][d3]  (layouts of hdg_recover)
 * Workspace: hdg_project_hdg_workspace_size bytes (the face moments, [nfc][4][d2]).
 * Errors: HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE, HDG_ERR_UNSUPPORTED_DEGREE. */
hdg_status hdg_project_hdg_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes);
hdg_status hdg_project_hdg(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_tau, const double* d_qu_vol,
                           const double* d_qu_face, double* d_Pq, double* d_Pu, void* d_ws, size_t ws_bytes,
                           void* stream);
/* Squared norms behind eq 10.2, into d_out double[4] (device): ||Pi u - u_h||^2_Omega,
 * ||u||^2_Omega, ||P u - uhat_h||_h^2 and ||u||_h^2 with ||v||_h^2 = sum_e |e| ||v||_e^2, so
 * that eps_u = sqrt(out[0] / out[1]) and eps_uhat = sqrt(out[2] / out[3]).
 *   d_Pu, d_uh  double [nelt][d3]   (hdg_project_hdg's Pi u, hdg_recover's u)
 *   d_Puhat, d_uhat double [nfc][d2] (hdg_project_trace of u over all faces, the solution)
 *   d_u_vol   double [nelt][nqd], d_u_face double [nfc][nqd2]: u at the quadrature points
 *             (either may be NULL: its norm is then 0)
 * The norms of the discrete differences use the orthonormal bases (|K| sum_i d_i^2 and
 * |e| sum_i d_i^2); those of u use the quadrature rules of disc.  Fixed-order reductions
 * (bitwise reproducible).  Workspace: hdg_superconvergence_norms_workspace_size bytes. */
hdg_status hdg_superconvergence_norms_workspace_size(const hdg_mesh* mesh, size_t* bytes);
hdg_status hdg_superconvergence_norms(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_Pu,
                                      const double* d_uh, const double* d_u_vol, const double* d_Puhat,
                                      const double* d_uhat, const double* d_u_face, double* d_out, void* d_ws,
                                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------
 * Condensation with FP32 local factorisations and FP64 iterative refinement (degrees
 * 1..3; eq 5.1-5.6, scatter of eq 6.5).
 *
 * X = A1^{-1} [A2 | Af] (eq 5.2-5.4) is computed by refinement X += P(B - A1 X).  The
 * residual uses A1's block structure and runs in FP64; P is the block elimination of A1
 * (M, and the Schur complement S = Mc + tauPP + sum_s C_s M^{-1} C_s^T) with FP32
 * Cholesky factors, applied on the FP32 matrix cores.  Sweeps stop once every column of
 * the right-hand side [A2 | Af] has settled (its correction at most 1e-15 of that column of
 * X, or no longer shrinking by half while below 1e-12 of it: the FP64 rounding floor), or
 * at max_sweeps (1..20).  Then C^K = A3 X_2 + tauDD and
 * Cf^K = A3 X_f (FP64) are scattered into H and F exactly as by hdg_assemble_condense.
 *   d_X       double [nelt][4 d3][4 d2 + 1]  X, kept for hdg_recover_ir (may be NULL);
 *             hdg_ir_store_len gives 4 d3 (4 d2 + 1)
 *   d_sweeps  int32 [nelt]  sweeps used per element (may be NULL); max_sweeps + 1 marks an
 *             element whose refinement had not met the bound after max_sweeps sweeps (its
 *             outputs are written all the same, at the accuracy reached)
 * Errors: HDG_ERR_UNSUPPORTED_DEGREE (k = 0 or 4), HDG_ERR_INVALID_ARG, HDG_ERR_SINGULAR (as
 * for hdg_assemble_condense).
 * ------------------------------------------------------------------------------ */
hdg_status hdg_ir_store_len(const hdg_disc* disc, int64_t* n);
hdg_status hdg_assemble_condense_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                    const double* d_c, const double* d_f, const double* d_tau, double* d_H,
                                    double* d_F, double* d_X, int max_sweeps, int32_t* d_sweeps, void* stream);
/* Per-element C^K [n][m][m], Cf^K [n][m] and (optional) X [n][4 d3][m + 1] of the listed
 * elements from the same refined local solve, instead of the scatter (for tests). */
hdg_status hdg_export_local_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa, const double* d_c,
                               const double* d_f, const double* d_tau, const int32_t* d_elems, int64_t n, double* d_C,
                               double* d_Cf, double* d_X, int max_sweeps, void* stream);
/* Reconstruction from the stored X: [q; u] = X_f - X_2 uhat_K (Section 6), degrees 0..4 (X
 * from hdg_assemble_condense_ir or hdg_assemble_condense_cd).  Outputs as in hdg_recover; the
 * postprocess is hdg_postprocess. */
hdg_status hdg_recover_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_X, const double* d_uhat,
                          double* d_q, double* d_u, void* stream);

/* ------------------------------------------------------------------------------
 * Convection-diffusion (Section 9, "Matrices for convection-diffusion problems"; the
 * element blocks of eq 9.1 with variable coefficients), degrees 0..3.
 *   kappa^{-1} q + grad u = 0,  div(q + beta u) + c u = f,
 * the numerical total flux q.nu + (beta.nu) uhat + tau (u - uhat) on every element boundary,
 * u = u_D on Dirichlet faces and, on Neumann faces, the total outward flux given:
 * -(q + beta u).nu = g_N . nu (hdg_boundary's g_N is then kappa grad u - beta u).  The local
 * matrices are those of the diffusion element plus: -sum_s E_s^T in the u block of A1
 * (E_s[i][j] = int_K beta_s P_i d_s P_j), +(beta.n DP_l)^T in the u rows of A2, and
 * -(beta.n DD_l) on the diagonal blocks of C^K (int_{e_l} (beta.nu) D_i P_j and D_i D_j).
 * The method is stable when tau >= beta.nu / 2 on every face and c + div(beta) / 2 >= 0;
 * the caller ensures it (and a unique solution: a Dirichlet face, or c + div(beta) / 2 > 0
 * somewhere).  H is then not symmetric: solve with hdg_solve_gmres.
 *
 * hdg_elem_face_qp_coords: the points phi_l^K(qhat_r) of each element's own parametrisation
 * of its four faces (reference face l of eq 2.5 mapped by F_K):
 *   d_xyz double [nelt][4][nqd2][3]; the caller evaluates beta there.
 * hdg_assemble_condense_cd:
 *   d_kappa, d_c, d_f  double [nelt][nqd]        at the points of hdg_qp_coords
 *   d_beta_vol         double [nelt][nqd][3]     beta at the points of hdg_qp_coords
 *   d_beta_face        double [nelt][4][nqd2][3] beta at the points of hdg_elem_face_qp_coords
 *   d_tau              double [nelt][4]
 * Outputs: d_H [nnzb][d2][d2] (every block written, row-major, not symmetric), d_F [nfc][d2],
 * d_X [nelt][4 d3][4 d2 + 1] (may be NULL) X = A1^{-1} [A2 | Af] for hdg_recover_ir.
 * The element's u Schur complement is factored by LU without pivoting (its symmetric part is
 * positive definite under the stability condition).  Errors: HDG_ERR_INVALID_ARG,
 * HDG_ERR_UNSUPPORTED_DEGREE (k = 4).
 * hdg_export_local_cd: C^K [n][m][m], Cf^K [n][m] and (optional) X [n][4 d3][m + 1] of the
 * listed elements instead of the scatter (for tests). */
hdg_status hdg_elem_face_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, double* d_xyz, void* stream);
hdg_status hdg_assemble_condense_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                    const double* d_c, const double* d_f, const double* d_beta_vol,
                                    const double* d_beta_face, const double* d_tau, double* d_H, double* d_F,
                                    double* d_X, void* stream);
hdg_status hdg_export_local_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa, const double* d_c,
                               const double* d_f, const double* d_beta_vol, const double* d_beta_face,
                               const double* d_tau, const int32_t* d_elems, int64_t n, double* d_C, double* d_Cf,
                               double* d_X, void* stream);

/* Restarted GMRES(restart) for the non-symmetric trace system after hdg_boundary (the paper
 * leaves the solver open): right preconditioning by the inverses of the d2 x d2 diagonal
 * blocks (Gauss-Jordan with partial pivoting), classical Gram-Schmidt with selective
 * reorthogonalisation,
 * fixed-order reductions (the same bits on every run).  The host solves the small
 * least-squares problem (Givens rotations) and reads one short vector per iteration; every
 * cycle starts from the true FP64 residual b - H x, and the solve ends when
 * ||b - H x|| <= rtol ||b|| or after max_iter inner iterations.
 *   d_uhat  in: initial guess (Dirichlet values set by hdg_boundary); out: the solution
 *   restart 1..64;  workspace of hdg_solve_gmres_workspace_size bytes, caller-owned
 *   info->iterations = inner iterations, info->outer = cycles, info->rel_residual the
 *   true relative residual, info->fell_back = the number of Arnoldi steps that took a second
 *   Gram-Schmidt pass (taken when the first left less than 1e-3 of ||w||).
 * Errors: HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE, HDG_ERR_NOT_CONVERGED (the solution at
 * max_iter is still written). */
hdg_status hdg_solve_gmres_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, int restart, size_t* ws_bytes);
hdg_status hdg_solve_gmres(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, const double* d_b,
                           double* d_uhat, double rtol, int max_iter, int restart, hdg_solve_info* info, void* d_ws,
                           size_t ws_bytes, void* stream);

/* BiCGStab (van der Vorst's stabilised bi-conjugate gradients) for the same non-symmetric
 * systems, right-preconditioned by the same block-Jacobi inverses: two products with H per
 * iteration and no restart.  The scalars stay on the device; the host reads ||r||^2 every
 * check_every iterations and accepts the iterate on the recomputed FP64 residual
 * ||b - H x|| <= rtol ||b|| (otherwise the residual is replaced by the true one and the
 * iteration starts again from x).  A breakdown (a non-finite residual) restarts from the
 * last checked iterate.  info->iterations = iterations, info->outer = restarts,
 * info->rel_residual = the true relative residual.  Workspace of
 * hdg_solve_bicgstab_workspace_size bytes, caller-owned.
 * Errors: HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE, HDG_ERR_NOT_CONVERGED. */
hdg_status hdg_solve_bicgstab_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* ws_bytes);
hdg_status hdg_solve_bicgstab(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, const double* d_b,
                              double* d_uhat, double rtol, int max_iter, int check_every, hdg_solve_info* info,
                              void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------
 * Learned face-graph preconditioner for eq 6.5 (the paper leaves the solver open).
 *
 * With H_ii = L_i L_i^T and Hs_ij = L_i^{-1} H_ij L_j^{-T} (block-Jacobi scaling), the
 * preconditioner is M^{-1} = L^{-T} G^T G L^{-1} with G = B (I + N), N strictly block-lower
 * on the pattern of H and B block diagonal with lower-triangular d2 x d2 blocks of positive
 * diagonal.  It is SPD for every N and B.  A message-passing network over the faces (FP32;
 * nodes = faces, edges = off-diagonal blocks of H) predicts N and B.  Its node features are
 * the face type, the log area and the row energy of Hs; its edge features are the entries
 * of Hs_ij.  The layers are
 *     X = relu(W0 a + c0), E = relu(We b + ce),
 *     M_ij = relu(Wm_l [X_i; X_j; E_ij] + cm_l), X_i += relu(Wu_l [X_i; sum_j M_ij] + cu_l),
 * and the two heads are
 *     N_ij = -Hs_ij + reshape(Wo [X_i; X_j; E_ij] + co)   (j < i, no Dirichlet face),
 *     beta_i = Wb X_i + cb   (fb = d2 (d2 + 1) / 2 values; zero on Dirichlet faces),
 * with B_i[a][a] = exp(beta_i[a]) and B_i[a][b] = beta_i[d2 + a (a - 1) / 2 + b] for b < a.
 * Zero heads give the first-order factor G = I - tril(Hs).  The parameters form one FP32
 * vector in the order W0, c0, We, ce, (Wm_l, cm_l, Wu_l, cu_l) for l = 1..L, Wo, co, Wb,
 * cb; matrices are row-major (output, input).
 * Training objective: the logarithm of the Kaporin number (tr/n) / det^{1/n} of G Hs G^T,
 * which bounds the PCG iteration count.  det(G Hs G^T) = det(B)^2 det(Hs), so up to a
 * constant
 *     loss = log T - (2/n) sum_i sum_a beta_i[a],
 *     T = 1/(p n) sum_z (G^T z)^T Hs (G^T z)   over p probe vectors z, n = nfc d2.
 * Every array is caller-owned device memory.  No call allocates, and every reduction
 * has a fixed order.
 * ------------------------------------------------------------------------------ */
typedef struct {
  int d2;       /* block size: 1, 3, 6, 10 or 15 (degree 0..4) */
  int hidden;   /* channels, 1..64 */
  int layers;   /* message-passing layers, 0..8 */
} hdg_gnn_shape;

typedef struct {
  float* Hs;        /* [nnzb][d2][d2]  scaled blocks (diagonal blocks: identity) */
  float* Linv;      /* [nfc][d2][d2]   L_i^{-1} (lower triangular) */
  float* node;      /* [nfc][5]        node features */
  int32_t* erow;    /* [nnzb]          block row of each stored block */
  int32_t* mirror;  /* [nnzb]          position of the transposed block */
} hdg_gnn_graph;

hdg_status hdg_gnn_param_count(const hdg_gnn_shape* shape, int64_t* n);
/* Graph of one system from H after hdg_boundary (Dirichlet rows are the identity).
 * Workspace: hdg_gnn_graph_workspace_size bytes (FP64 factors).  Errors:
 * HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE, HDG_ERR_UNSUPPORTED_DEGREE. */
hdg_status hdg_gnn_graph_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes);
hdg_status hdg_gnn_build_graph(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, hdg_gnn_graph* graph,
                               void* d_ws, size_t ws_bytes, void* stream);
/* Activations and temporaries of forward / backward for nprobe probe vectors. */
hdg_status hdg_gnn_workspace_size(const hdg_gnn_shape* shape, const hdg_mesh* mesh, int nprobe, size_t* bytes);
/* d_N [nnzb][d2][d2]: N_ij on the lower blocks (j < i) without Dirichlet faces, zero on the
 * other lower blocks and on the diagonal, and N_ij^T at each mirrored upper position (j, i)
 * (so that the transposed sweep of the preconditioner reads block rows);
 * d_B [nfc][d2 (d2 + 1) / 2]: beta of every face (zero on Dirichlet faces). */
hdg_status hdg_gnn_forward(const hdg_gnn_shape* shape, const float* d_params, const hdg_mesh* mesh,
                           const hdg_gnn_graph* graph, float* d_N, float* d_B, void* d_ws, size_t ws_bytes,
                           void* stream);
/* Forward, the loss and its gradient: d_probes [nprobe][nfc][d2] (drawn by the caller),
 * d_N and d_B as from hdg_gnn_forward, d_loss one double (device), d_grad [param_count]
 * (NULL: loss only). */
hdg_status hdg_gnn_loss_grad(const hdg_gnn_shape* shape, const float* d_params, const hdg_mesh* mesh,
                             const hdg_gnn_graph* graph, const float* d_probes, int nprobe, float* d_N, float* d_B,
                             double* d_loss, float* d_grad, void* d_ws, size_t ws_bytes, void* stream);
/* z = M^{-1} r = L^{-T} G^T G L^{-1} r with G = B (I + N): the learned preconditioner as
 * hdg_solve applies it (precond = 1), FP64 vectors with FP32 factors and FP64 accumulation.
 *   d_N [nnzb][d2][d2] and d_B [nfc][d2 (d2 + 1) / 2] (hdg_gnn_forward; d_B may be NULL for
 *   B = I), d_Linv [nfc][d2][d2] (the graph), d_r and d_z double [nfc][d2] (distinct arrays).
 * Workspace: nfc d2 doubles.  Errors: HDG_ERR_INVALID_ARG, HDG_ERR_WORKSPACE. */
hdg_status hdg_gnn_precond_apply(const hdg_disc* disc, const hdg_mesh* mesh, const float* d_N, const float* d_B,
                                 const float* d_Linv, const double* d_r, double* d_z, void* d_ws, size_t ws_bytes,
                                 void* stream);
/* Checkpoints of the parameter vector in the safetensors layout: an 8-byte little-endian
 * header length, a JSON header {"__metadata__": {string: string}, "params": {"dtype": "F32",
 * "shape": [n], "data_offsets": [0, 4 n]}}, then n little-endian FP32 words.  The metadata
 * holds the shape as "d2", "hidden", "layers" and any caller pairs.  Host memory only.
 *   hdg_gnn_save: h_params [n] (n = hdg_gnn_param_count(shape)), nmeta caller pairs
 *   hdg_gnn_load_info: the shape and n of a file;  hdg_gnn_load: its parameters into h_params [n]
 *   hdg_gnn_checkpoint_meta: the value of one metadata key; *len its length, out (may be NULL)
 *     receives at most cap - 1 bytes and a terminating zero
 * Errors: HDG_ERR_INVALID_ARG (I/O failure, malformed file, count or shape mismatch). */
hdg_status hdg_gnn_save(const char* path, const hdg_gnn_shape* shape, const float* h_params, int64_t n,
                        const char* const* meta_keys, const char* const* meta_values, int nmeta);
hdg_status hdg_gnn_load_info(const char* path, hdg_gnn_shape* shape, int64_t* n);
hdg_status hdg_gnn_load(const char* path, float* h_params, int64_t n);
hdg_status hdg_gnn_checkpoint_meta(const char* path, const char* key, char* out, size_t cap, size_t* len);
/* One Adam step (step = 1, 2, ...) on n parameters. */
hdg_status hdg_gnn_adam(int64_t n, float* d_params, const float* d_grad, float* d_m, float* d_v, int step, float lr,
                        float beta1, float beta2, float eps, void* stream);

/* ------------------------------------------------------------------------------
 * Batched condensation of many independent meshes of mixed degree in one launch.
 *
 * Each mesh of the batch gets exactly what hdg_assemble_condense gives it (H, F and the
 * factor store, bit for bit); the element work is that of Sections 3-6 (eq 5.5-5.6) and
 * the scatter of eq 6.5, cut into work units (groups of four elements for k = 1..3,
 * single elements for k = 0 and 4) and swept by one persistent kernel per degree; degrees
 * 0..4 (hdg_batch_create returns HDG_ERR_UNSUPPORTED_DEGREE for a mesh of degree 5 or 6).
 *
 * hdg_batch_create copies the item list and the mesh structs; the discs, the mesh arrays,
 * the coefficient arrays and the outputs stay owned by the caller and must outlive the
 * batch.  Two items must not share an output array (their writes would race).  It
 * allocates the device work lists, one stream per degree and the capture objects
 * (set-up, not a compute call).  Errors: HDG_ERR_INVALID_ARG (n < 1, NULL arrays, an
 * unexpanded mesh, nq != k + 2), HDG_ERR_SINGULAR (an item as in hdg_assemble_condense;
 * checked here, on the null stream), HDG_ERR_DEVICE.
 * ------------------------------------------------------------------------------ */
typedef struct {
  const hdg_disc* disc;      /* degree and tables (nq = k + 2) */
  const hdg_mesh* mesh;      /* expanded mesh */
  const double* d_kappa;     /* double [nelt][nqd]  as in hdg_assemble_condense */
  const double* d_c;         /* double [nelt][nqd] */
  const double* d_f;         /* double [nelt][nqd] */
  const double* d_tau;       /* double [nelt][4] */
  double* d_H;               /* double [nnzb][d2][d2]  output */
  double* d_F;               /* double [nfc][d2]       output */
  double* d_factors;         /* double [nelt][factor_len] output, may be NULL */
} hdg_batch_item;

/* Launch shape of one degree's persistent kernel: the grid is workgroups_per_cu times
 * the number of compute units (at most the number of work units); xcd_remap = 1 hands
 * each of the eight XCDs a contiguous run of work units per sweep; waves_per_element is
 * the workgroup size, in wavefronts, of the per-element kernel of k = 0 and 4 (1, 2, 4
 * or 8; must be 1 for the four-elements-per-wavefront kernels of k = 1..3).
 * A new batch starts from the library-wide shape of hdg_get_launch_config. */
typedef struct {
  int workgroups_per_cu;     /* 1..64 */
  int xcd_remap;             /* 0 or 1 */
  int waves_per_element;     /* 1, 2, 4, 8 */
} hdg_tile_config;

/* Library-wide launch shape of the condensation of degree k, used by hdg_assemble_condense
 * and hdg_export_local and as the starting shape of new batches (defaults: k = 1..3
 * {4, 1, 1}, k = 4 {2, 1, 4}, k = 0 {2, 0, 1}, k = 5, 6 {1, 0, 4}; degrees 5 and 6 use
 * workgroups_per_cu and xcd_remap only, and their workspace size follows workgroups_per_cu).
 * Every shape gives the same results bit for bit.  Not synchronised with calls running in
 * other threads.  Errors: HDG_ERR_INVALID_ARG. */
hdg_status hdg_set_launch_config(int k, const hdg_tile_config* cfg);
hdg_status hdg_get_launch_config(int k, hdg_tile_config* cfg);

typedef struct hdg_batch hdg_batch;

hdg_status hdg_batch_create(int n, const hdg_batch_item* items, hdg_batch** out);
hdg_status hdg_batch_destroy(hdg_batch* batch);
/* Number of meshes and elements of degree k in the batch. */
hdg_status hdg_batch_info(const hdg_batch* batch, int k, int64_t* nmesh, int64_t* nelt);
hdg_status hdg_batch_set_config(hdg_batch* batch, int k, const hdg_tile_config* cfg);
hdg_status hdg_batch_get_config(const hdg_batch* batch, int k, hdg_tile_config* cfg);
/* Eager form: per degree (highest first) zero the diagonal blocks of H and F of its
 * meshes, then run the persistent kernel; all on `stream`. */
hdg_status hdg_batch_condense(hdg_batch* batch, void* stream);
/* (Re)records the same work, in the same order, as one hipGraph (the per-degree parts
 * are chained, not parallel: each persistent kernel is sized for the whole chip); called
 * by hdg_batch_launch when no graph exists or the configuration changed. */
hdg_status hdg_batch_capture(hdg_batch* batch);
/* One graph launch of the whole batch on `stream`. */
hdg_status hdg_batch_launch(hdg_batch* batch, void* stream);

/* Autotuner for degree k on this batch: times every candidate shape (k = 1..3:
 * workgroups_per_cu in {1, 2, 4, 8, 16} x xcd_remap in {0, 1}; k = 0, 4: workgroups_per_cu
 * in {1, 2} x xcd_remap x waves_per_element in {1, 2, 4, 8}), each once to warm up and then `reps` times on
 * `stream` (the batch's degree-k outputs are overwritten with identical values), keeps the
 * fastest in the batch and returns it.  ncand, cands [16] and cand_ms [16] may be NULL;
 * else they receive every candidate and its mean time (ms).  Synchronises the stream.
 * Errors: HDG_ERR_INVALID_ARG (no mesh of degree k, reps < 1), HDG_ERR_DEVICE. */
hdg_status hdg_autotune(hdg_batch* batch, int k, int reps, hdg_tile_config* best, double* best_ms, int* ncand,
                        hdg_tile_config* cands, double* cand_ms, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
