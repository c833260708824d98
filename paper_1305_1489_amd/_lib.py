"""ctypes binding of libhdg (include/hdg.h).

Argument marshalling only: every function here has the name of the C call it wraps,
takes torch tensors (device memory) and plain Python values, allocates caller-owned
outputs with torch where the C call expects them, and raises :class:`HdgError` on a
non-zero status.  All arithmetic happens inside the library's HIP kernels.  The
library must have been built (``python -m paper_1305_1489_amd.build``); there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

STATUS = {0: "HDG_OK", 1: "HDG_ERR_INVALID_ARG", 2: "HDG_ERR_UNSUPPORTED_DEGREE", 3: "HDG_ERR_MESH_ORIENTATION",
          4: "HDG_ERR_MESH_NONCONFORMING", 5: "HDG_ERR_BOUNDARY_UNLISTED", 6: "HDG_ERR_BOUNDARY_INVALID",
          7: "HDG_ERR_TAU_ZERO", 8: "HDG_ERR_WORKSPACE", 9: "HDG_ERR_DEVICE", 10: "HDG_ERR_NOT_CONVERGED",
          11: "HDG_ERR_SINGULAR"}

EXPORTS = ["hdg_last_error", "hdg_max_degree", "hdg_mesh_sizes", "hdg_mesh_expand", "hdg_disc_create",
           "hdg_disc_destroy", "hdg_disc_get_info", "hdg_disc_table", "hdg_reference_table", "hdg_qp_coords", "hdg_face_qp_coords",
           "hdg_assemble_condense", "hdg_condense_workspace_size", "hdg_assemble_condense_ws", "hdg_check_tau", "hdg_export_local", "hdg_boundary",
           "hdg_solve_workspace_size", "hdg_solve", "hdg_recover", "hdg_postprocess", "hdg_batch_create",
           "hdg_batch_destroy", "hdg_batch_info", "hdg_batch_set_config", "hdg_batch_get_config",
           "hdg_batch_condense", "hdg_batch_capture", "hdg_batch_launch", "hdg_autotune", "hdg_set_launch_config",
           "hdg_get_launch_config", "hdg_gnn_param_count", "hdg_gnn_graph_workspace_size", "hdg_gnn_build_graph",
           "hdg_gnn_workspace_size", "hdg_gnn_forward", "hdg_gnn_loss_grad", "hdg_gnn_adam", "hdg_ir_store_len",
           "hdg_assemble_condense_ir", "hdg_recover_ir", "hdg_export_local_ir", "hdg_condense_noalloc_capacity",
           "hdg_assemble_condense_noalloc", "hdg_set_kernel_timer", "hdg_project_trace",
           "hdg_project_hdg_workspace_size", "hdg_project_hdg", "hdg_superconvergence_norms_workspace_size",
           "hdg_superconvergence_norms", "hdg_assemble_condense_bdm", "hdg_gnn_precond_apply",
           "hdg_elem_face_qp_coords", "hdg_assemble_condense_cd", "hdg_export_local_cd",
           "hdg_solve_gmres_workspace_size", "hdg_solve_gmres", "hdg_gnn_save", "hdg_gnn_load_info", "hdg_gnn_load",
           "hdg_gnn_checkpoint_meta", "hdg_solve_bicgstab_workspace_size", "hdg_solve_bicgstab"]


class HdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class hdg_mesh(C.Structure):
    _fields_ = [("nver", C.c_int64), ("nelt", C.c_int64), ("ndir", C.c_int64), ("nneu", C.c_int64),
                ("nfc", C.c_int64), ("nnzb", C.c_int64)] + [(n, C.c_void_p) for n in (
                    "d_coords", "d_elements", "d_dirichlet", "d_neumann", "d_faces", "d_ftype", "d_dirfaces",
                    "d_neufaces", "d_facebyele", "d_perm", "d_volume", "d_area", "d_normals", "d_face_elem",
                    "d_row_ptr", "d_col_idx", "d_diag", "d_slot")]


class hdg_disc_info(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("k", "nq", "d3", "d2", "m", "d3p", "nqd", "nqd2", "factor_len")]


class hdg_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int), ("precision", C.c_int),
                ("precond", C.c_int), ("d_pre_N", C.c_void_p), ("d_pre_Linv", C.c_void_p),
                ("d_pre_B", C.c_void_p)]


class hdg_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer", C.c_int), ("rel_residual", C.c_double), ("fell_back", C.c_int)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhdg is not built ({LIB_PATH} missing): run python -m paper_1305_1489_amd.build")
        L = C.CDLL(LIB_PATH)
        L.hdg_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("hdg_last_error",):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise HdgError(code, lib().hdg_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(x, dtype, device):
    return torch.as_tensor(x, dtype=dtype).to(device).contiguous()


# ----------------------------------------------------------------------------- mesh
class Mesh:
    """Owns the device arrays of an expanded mesh and the hdg_mesh struct that points at them."""

    def __init__(self, coords, elements, dirichlet, neumann, device="cuda"):
        self.device = torch.device(device)
        self.coords = _dev(coords, torch.float64, self.device).reshape(-1, 3)
        self.elements = _dev(elements, torch.int32, self.device).reshape(-1, 4)
        self.dirichlet = _dev(dirichlet, torch.int32, self.device).reshape(-1, 3)
        self.neumann = _dev(neumann, torch.int32, self.device).reshape(-1, 3)
        m = hdg_mesh()
        m.nver, m.nelt = self.coords.shape[0], self.elements.shape[0]
        m.ndir, m.nneu = self.dirichlet.shape[0], self.neumann.shape[0]
        self.struct = m
        self.ws_bytes = hdg_mesh_sizes(self)
        nfc, nelt, nnzb = m.nfc, m.nelt, m.nnzb
        i32 = dict(dtype=torch.int32, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.faces = torch.zeros((nfc, 3), **i32)
        self.ftype = torch.zeros(nfc, **i32)
        self.dirfaces = torch.zeros(max(m.ndir, 1), **i32)
        self.neufaces = torch.zeros(max(m.nneu, 1), **i32)
        self.facebyele = torch.zeros((nelt, 4), **i32)
        self.perm = torch.zeros((nelt, 4), **i32)
        self.volume = torch.zeros(nelt, **f64)
        self.area = torch.zeros(nfc, **f64)
        self.normals = torch.zeros((nelt, 4, 3), **f64)
        self.face_elem = torch.zeros((nfc, 2), **i32)
        self.row_ptr = torch.zeros(nfc + 1, **i32)
        self.col_idx = torch.zeros(nnzb, **i32)
        self.diag = torch.zeros(nfc, **i32)
        self.slot = torch.zeros((nelt, 16), **i32)
        for name in ("coords", "elements", "dirichlet", "neumann", "faces", "ftype", "dirfaces", "neufaces",
                     "facebyele", "perm", "volume", "area", "normals", "face_elem", "row_ptr", "col_idx", "diag",
                     "slot"):
            setattr(m, "d_" + name, _ptr(getattr(self, name)).value)

    @property
    def nelt(self):
        return self.struct.nelt

    @property
    def nfc(self):
        return self.struct.nfc

    @property
    def nnzb(self):
        return self.struct.nnzb

    @property
    def ndir(self):
        return self.struct.ndir

    @property
    def nneu(self):
        return self.struct.nneu


def hdg_mesh_sizes(mesh: Mesh) -> int:
    ws = C.c_size_t(0)
    _check(lib().hdg_mesh_sizes(C.byref(mesh.struct), C.byref(ws)))
    return ws.value


def hdg_mesh_expand(coords, elements, dirichlet, neumann, device="cuda", stream=None) -> Mesh:
    mesh = Mesh(coords, elements, dirichlet, neumann, device)
    ws = torch.empty(max(mesh.ws_bytes, 8), dtype=torch.uint8, device=mesh.device)
    _check(lib().hdg_mesh_expand(C.byref(mesh.struct), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream)))
    return mesh


# ----------------------------------------------------------------------------- discretisation
class Disc:
    def __init__(self, handle):
        self.handle = handle
        info = hdg_disc_info()
        _check(lib().hdg_disc_get_info(handle, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in hdg_disc_info._fields_}

    def __getattr__(self, item):
        info = self.__dict__.get("info")
        if info is not None and item in info:
            return info[item]
        raise AttributeError(item)

    def __del__(self):
        h = self.__dict__.get("handle")
        if h and _lib is not None:
            _lib.hdg_disc_destroy(h)
            self.handle = None


def hdg_disc_create(k: int, nq: int = 0) -> Disc:
    h = C.c_void_p()
    _check(lib().hdg_disc_create(C.c_int(k), C.c_int(nq), C.byref(h)))
    return Disc(h)


def hdg_disc_get_info(disc: Disc) -> dict:
    return dict(disc.info)


def hdg_disc_table(disc: Disc, name: str) -> np.ndarray:
    n = C.c_int64(0)
    _check(lib().hdg_disc_table(disc.handle, name.encode(), None, C.byref(n)))
    out = np.zeros(n.value)
    _check(lib().hdg_disc_table(disc.handle, name.encode(), out.ctypes.data_as(C.c_void_p), C.byref(n)))
    return out


def hdg_reference_table(k: int, name: str, nq: int = 0) -> np.ndarray:
    """Host-only table build (no device needed)."""
    n = C.c_int64(0)
    _check(lib().hdg_reference_table(C.c_int(k), C.c_int(nq), name.encode(), None, C.byref(n)))
    out = np.zeros(n.value)
    _check(lib().hdg_reference_table(C.c_int(k), C.c_int(nq), name.encode(), out.ctypes.data_as(C.c_void_p),
                                     C.byref(n)))
    return out


def hdg_max_degree() -> int:
    return lib().hdg_max_degree()


# ----------------------------------------------------------------------------- compute calls
def hdg_qp_coords(disc: Disc, mesh: Mesh, out=None, stream=None):
    if out is None:
        out = torch.empty((mesh.nelt, disc.nqd, 3), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_qp_coords(disc.handle, C.byref(mesh.struct), _ptr(out), _stream(stream)))
    return out


def hdg_face_qp_coords(disc: Disc, mesh: Mesh, faces, out=None, stream=None):
    faces = _dev(faces, torch.int32, mesh.device).reshape(-1)
    n = faces.numel()
    if out is None:
        out = torch.empty((n, disc.nqd2, 3), dtype=torch.float64, device=mesh.device)
    if n:
        _check(lib().hdg_face_qp_coords(disc.handle, C.byref(mesh.struct), _ptr(faces), C.c_int64(n), _ptr(out),
                                        _stream(stream)))
    return out


def hdg_check_tau(mesh: Mesh, tau, stream=None):
    _check(lib().hdg_check_tau(C.byref(mesh.struct), _ptr(tau), _stream(stream)))


def hdg_assemble_condense(disc: Disc, mesh: Mesh, kappa, c, f, tau, H=None, F=None, factors=None, stream=None):
    d2 = disc.d2
    if H is None:
        H = torch.empty((mesh.nnzb, d2, d2), dtype=torch.float64, device=mesh.device)
    if F is None:
        F = torch.empty((mesh.nfc, d2), dtype=torch.float64, device=mesh.device)
    if factors is None:
        factors = torch.empty((mesh.nelt, disc.factor_len), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_assemble_condense(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(tau),
                                       _ptr(H), _ptr(F), _ptr(factors), _stream(stream)))
    return H, F, factors


def hdg_condense_workspace_size(disc: Disc, mesh: Mesh) -> int:
    n = C.c_size_t(0)
    _check(lib().hdg_condense_workspace_size(disc.handle, C.byref(mesh.struct), C.byref(n)))
    return n.value


def hdg_assemble_condense_ws(disc: Disc, mesh: Mesh, kappa, c, f, tau, H, F, factors, ws=None, stream=None):
    """hdg_assemble_condense without atomics (same bits); ws: a uint8 device tensor of at least
    hdg_condense_workspace_size bytes, allocated here when None."""
    need = hdg_condense_workspace_size(disc, mesh)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=mesh.device)
    _check(lib().hdg_assemble_condense_ws(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(tau),
                                          _ptr(H), _ptr(F), _ptr(factors), _ptr(ws), C.c_size_t(ws.numel()),
                                          _stream(stream)))
    return H, F, factors


def hdg_set_kernel_timer(kernel, ev_start=None, ev_stop=None):
    """Bracket launches of the named kernel with the caller's hipEvent_t handles (ints or
    c_void_p); kernel=None switches the timer off."""
    _check(lib().hdg_set_kernel_timer(None if kernel is None else kernel.encode(), C.c_void_p(ev_start),
                                      C.c_void_p(ev_stop)))


def hdg_condense_noalloc_capacity() -> int:
    n = C.c_size_t(0)
    _check(lib().hdg_condense_noalloc_capacity(C.byref(n)))
    return n.value


def hdg_assemble_condense_noalloc(disc: Disc, mesh: Mesh, kappa, c, f, tau, H, F, factors, stream=None):
    """hdg_assemble_condense_ws with the library's static device workspace (no allocation)."""
    _check(lib().hdg_assemble_condense_noalloc(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f),
                                               _ptr(tau), _ptr(H), _ptr(F), _ptr(factors), _stream(stream)))
    return H, F, factors


def hdg_project_trace(disc: Disc, mesh: Mesh, vals, out=None, stream=None):
    """eq 9.12 for the fields vals [n][nqd2][ncomp] at the face points of n faces ->
    [n][ncomp][d2]."""
    if vals.dim() == 2:
        vals = vals.unsqueeze(-1)
    n, _, ncomp = vals.shape
    if out is None:
        out = torch.empty((n, ncomp, disc.d2), dtype=torch.float64, device=vals.device)
    _check(lib().hdg_project_trace(disc.handle, C.byref(mesh.struct), C.c_int64(n), C.c_int(ncomp), _ptr(vals),
                                   _ptr(out), _stream(stream)))
    return out


def hdg_project_hdg(disc: Disc, mesh: Mesh, tau, qu_vol, qu_face, Pq=None, Pu=None, ws=None, stream=None):
    """eq 9.13: (Pi q, Pi u) from (q, u) at the volume points [nelt][nqd][4] and the face
    points of every face [nfc][nqd2][4]."""
    n = C.c_size_t(0)
    _check(lib().hdg_project_hdg_workspace_size(disc.handle, C.byref(mesh.struct), C.byref(n)))
    if ws is None:
        ws = torch.empty(max(n.value, 8), dtype=torch.uint8, device=qu_vol.device)
    if Pq is None:
        Pq = torch.empty((mesh.nelt, 3, disc.d3), dtype=torch.float64, device=qu_vol.device)
    if Pu is None:
        Pu = torch.empty((mesh.nelt, disc.d3), dtype=torch.float64, device=qu_vol.device)
    _check(lib().hdg_project_hdg(disc.handle, C.byref(mesh.struct), _ptr(tau), _ptr(qu_vol), _ptr(qu_face),
                                 _ptr(Pq), _ptr(Pu), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream)))
    return Pq, Pu


def hdg_superconvergence_norms(disc: Disc, mesh: Mesh, Pu, uh, Puhat, uhat, u_vol=None, u_face=None, out=None,
                               ws=None, stream=None):
    """The four squared norms behind eq 10.2 as a device tensor of 4 doubles."""
    n = C.c_size_t(0)
    _check(lib().hdg_superconvergence_norms_workspace_size(C.byref(mesh.struct), C.byref(n)))
    if ws is None:
        ws = torch.empty(max(n.value, 8), dtype=torch.uint8, device=Pu.device)
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=Pu.device)
    _check(lib().hdg_superconvergence_norms(disc.handle, C.byref(mesh.struct), _ptr(Pu), _ptr(uh), _ptr(u_vol),
                                            _ptr(Puhat), _ptr(uhat), _ptr(u_face), _ptr(out), _ptr(ws),
                                            C.c_size_t(ws.numel()), _stream(stream)))
    return out


def hdg_assemble_condense_bdm(disc: Disc, mesh: Mesh, kappa, c, f, H, F, factors, ws=None, stream=None):
    """The hybridized BDM element (tau = 0, u in P_{k-1}) into H, F and the factor store."""
    need = hdg_condense_workspace_size(disc, mesh)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=mesh.device)
    _check(lib().hdg_assemble_condense_bdm(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(H),
                                           _ptr(F), _ptr(factors), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream)))
    return H, F, factors


def hdg_gnn_precond_apply(disc: Disc, mesh: Mesh, N, B, Linv, r, z=None, ws=None, stream=None):
    """z = L^{-T} G^T G L^{-1} r (G = B (I + N); B = None: the identity), as the learned PCG applies it."""
    if z is None:
        z = torch.empty_like(r)
    if ws is None:
        ws = torch.empty(mesh.nfc * disc.d2 * 8, dtype=torch.uint8, device=r.device)
    _check(lib().hdg_gnn_precond_apply(disc.handle, C.byref(mesh.struct), _ptr(N), _ptr(B), _ptr(Linv), _ptr(r),
                                       _ptr(z), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream)))
    return z


def hdg_export_local(disc: Disc, mesh: Mesh, kappa, c, f, tau, elems, stream=None):
    elems = _dev(elems, torch.int32, mesh.device).reshape(-1)
    n = elems.numel()
    m = disc.m
    Cm = torch.empty((n, m, m), dtype=torch.float64, device=mesh.device)
    Cf = torch.empty((n, m), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_export_local(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(tau),
                                  _ptr(elems), C.c_int64(n), _ptr(Cm), _ptr(Cf), _stream(stream)))
    return Cm, Cf


def hdg_boundary(disc: Disc, mesh: Mesh, uD, gN, H, F, uhat=None, stream=None):
    if uhat is None:
        uhat = torch.empty((mesh.nfc, disc.d2), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_boundary(disc.handle, C.byref(mesh.struct), _ptr(uD), _ptr(gN), _ptr(H), _ptr(F), _ptr(uhat),
                              _stream(stream)))
    return uhat


def hdg_solve_workspace_size(disc: Disc, mesh: Mesh, precision: int = 0) -> int:
    ws = C.c_size_t(0)
    _check(lib().hdg_solve_workspace_size(disc.handle, C.byref(mesh.struct), C.c_int(precision), C.byref(ws)))
    return ws.value


def hdg_solve(disc: Disc, mesh: Mesh, H, b, uhat, rtol=1e-10, max_iter=100000, check_every=10, precision=0,
              ws=None, stream=None, raise_on_fail=True, learned=None):
    """learned: None (block-Jacobi), or (N, B, graph) / (N, graph) from hdg_gnn_forward and
    hdg_gnn_build_graph (B = None: no block scaling)."""
    need = hdg_solve_workspace_size(disc, mesh, precision)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 8), dtype=torch.uint8, device=mesh.device)
    opts = hdg_solve_opts(rtol=rtol, max_iter=max_iter, check_every=check_every, precision=precision)
    if learned is not None:
        N, B, graph = learned if len(learned) == 3 else (learned[0], None, learned[1])
        opts.precond = 1
        opts.d_pre_N = N.data_ptr()
        opts.d_pre_B = B.data_ptr() if B is not None else None
        opts.d_pre_Linv = graph.Linv.data_ptr()
    info = hdg_solve_info()
    code = lib().hdg_solve(disc.handle, C.byref(mesh.struct), _ptr(H), _ptr(b), _ptr(uhat), C.byref(opts),
                           C.byref(info), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream))
    out = {"iterations": info.iterations, "outer": info.outer, "rel_residual": info.rel_residual, "status": code,
           "fell_back": bool(info.fell_back)}
    if code != 0 and raise_on_fail:
        _check(code)
    return out


def hdg_recover(disc: Disc, mesh: Mesh, kappa, tau, factors, uhat, q=None, u=None, ustar=None, postprocess=True,
                stream=None):
    if q is None:
        q = torch.empty((mesh.nelt, 3, disc.d3), dtype=torch.float64, device=mesh.device)
    if u is None:
        u = torch.empty((mesh.nelt, disc.d3), dtype=torch.float64, device=mesh.device)
    if postprocess and ustar is None:
        ustar = torch.empty((mesh.nelt, disc.d3p), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_recover(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(tau), _ptr(factors), _ptr(uhat),
                             _ptr(q), _ptr(u), _ptr(ustar) if postprocess else None, _stream(stream)))
    return q, u, (ustar if postprocess else None)


def hdg_postprocess(disc: Disc, mesh: Mesh, kappa, tau, q, u, ustar=None, stream=None, factors=None):
    """factors: the condensation's factor store (optional; the geometry is then read from it)."""
    if ustar is None:
        ustar = torch.empty((mesh.nelt, disc.d3p), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_postprocess(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(tau), _ptr(q), _ptr(u),
                                 _ptr(factors), _ptr(ustar), _stream(stream)))
    return ustar


# ----------------------------------------------------------------------------- batched condensation
class hdg_batch_item(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("disc", "mesh", "d_kappa", "d_c", "d_f", "d_tau", "d_H", "d_F",
                                          "d_factors")]


class hdg_tile_config(C.Structure):
    _fields_ = [("workgroups_per_cu", C.c_int), ("xcd_remap", C.c_int), ("waves_per_element", C.c_int)]


class Batch:
    """Owns an hdg_batch handle and keeps alive everything its work list points at."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        h = self.__dict__.get("handle")
        if h and _lib is not None:
            _lib.hdg_batch_destroy(h)
            self.handle = None


def hdg_batch_create(items) -> Batch:
    """items: sequence of dicts with keys disc, mesh, kappa, c, f, tau, H, F and optionally
    factors (tensors as for hdg_assemble_condense)."""
    arr = (hdg_batch_item * len(items))()
    keep = []
    for i, it in enumerate(items):
        for name in ("kappa", "c", "f", "tau", "H", "F"):
            t = it[name]
            if t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError(f"batch item {i}: {name} must be a contiguous float64 tensor")
        a = arr[i]
        a.disc = it["disc"].handle.value if isinstance(it["disc"].handle, C.c_void_p) else it["disc"].handle
        a.mesh = C.addressof(it["mesh"].struct)
        for name in ("kappa", "c", "f", "tau", "H", "F"):
            setattr(a, "d_" + name, it[name].data_ptr())
        fac = it.get("factors")
        a.d_factors = fac.data_ptr() if fac is not None else None
        keep.append(it)
    h = C.c_void_p()
    _check(lib().hdg_batch_create(C.c_int(len(items)), arr, C.byref(h)))
    return Batch(h, keep)


def hdg_batch_info(batch: Batch, k: int):
    nm, ne = C.c_int64(), C.c_int64()
    _check(lib().hdg_batch_info(batch.handle, C.c_int(k), C.byref(nm), C.byref(ne)))
    return nm.value, ne.value


def hdg_batch_set_config(batch: Batch, k: int, workgroups_per_cu: int, xcd_remap: int, waves_per_element: int = 1):
    cfg = hdg_tile_config(workgroups_per_cu, xcd_remap, waves_per_element)
    _check(lib().hdg_batch_set_config(batch.handle, C.c_int(k), C.byref(cfg)))


def hdg_batch_get_config(batch: Batch, k: int):
    cfg = hdg_tile_config()
    _check(lib().hdg_batch_get_config(batch.handle, C.c_int(k), C.byref(cfg)))
    return {"workgroups_per_cu": cfg.workgroups_per_cu, "xcd_remap": cfg.xcd_remap,
            "waves_per_element": cfg.waves_per_element}


def hdg_batch_condense(batch: Batch, stream=None):
    _check(lib().hdg_batch_condense(batch.handle, _stream(stream)))


def hdg_batch_capture(batch: Batch):
    _check(lib().hdg_batch_capture(batch.handle))


def hdg_batch_launch(batch: Batch, stream=None):
    _check(lib().hdg_batch_launch(batch.handle, _stream(stream)))


def hdg_autotune(batch: Batch, k: int, reps: int = 3, stream=None):
    best = hdg_tile_config()
    best_ms = C.c_double()
    nc = C.c_int()
    cands = (hdg_tile_config * 16)()
    cms = (C.c_double * 16)()
    _check(lib().hdg_autotune(batch.handle, C.c_int(k), C.c_int(reps), C.byref(best), C.byref(best_ms), C.byref(nc),
                              cands, cms, _stream(stream)))
    shape = lambda c: {"workgroups_per_cu": c.workgroups_per_cu, "xcd_remap": c.xcd_remap,
                       "waves_per_element": c.waves_per_element}
    return {"best": shape(best), "best_ms": best_ms.value,
            "candidates": [dict(shape(cands[i]), ms=cms[i]) for i in range(nc.value)]}


def hdg_set_launch_config(k: int, workgroups_per_cu: int, xcd_remap: int, waves_per_element: int = 1):
    cfg = hdg_tile_config(workgroups_per_cu, xcd_remap, waves_per_element)
    _check(lib().hdg_set_launch_config(C.c_int(k), C.byref(cfg)))


def hdg_get_launch_config(k: int):
    cfg = hdg_tile_config()
    _check(lib().hdg_get_launch_config(C.c_int(k), C.byref(cfg)))
    return {"workgroups_per_cu": cfg.workgroups_per_cu, "xcd_remap": cfg.xcd_remap,
            "waves_per_element": cfg.waves_per_element}


# ----------------------------------------------------------------------------- learned preconditioner
class hdg_gnn_shape(C.Structure):
    _fields_ = [("d2", C.c_int), ("hidden", C.c_int), ("layers", C.c_int)]


class hdg_gnn_graph(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("Hs", "Linv", "node", "erow", "mirror")]


class GnnGraph:
    """Owns the graph arrays of one system (hdg_gnn_build_graph)."""

    def __init__(self, nfc, nnzb, d2, device):
        f32 = dict(dtype=torch.float32, device=device)
        self.Hs = torch.zeros((nnzb, d2, d2), **f32)
        self.Linv = torch.zeros((nfc, d2, d2), **f32)
        self.node = torch.zeros((nfc, 5), **f32)
        self.erow = torch.zeros(nnzb, dtype=torch.int32, device=device)
        self.mirror = torch.zeros(nnzb, dtype=torch.int32, device=device)
        g = hdg_gnn_graph()
        for n in ("Hs", "Linv", "node", "erow", "mirror"):
            setattr(g, n, getattr(self, n).data_ptr())
        self.struct = g


def _shape(shape):
    return shape if isinstance(shape, hdg_gnn_shape) else hdg_gnn_shape(*shape)


def hdg_gnn_param_count(shape) -> int:
    n = C.c_int64()
    _check(lib().hdg_gnn_param_count(C.byref(_shape(shape)), C.byref(n)))
    return n.value


def hdg_gnn_build_graph(disc: Disc, mesh: Mesh, H, stream=None) -> GnnGraph:
    g = GnnGraph(mesh.nfc, mesh.nnzb, disc.d2, mesh.device)
    need = C.c_size_t()
    _check(lib().hdg_gnn_graph_workspace_size(disc.handle, C.byref(mesh.struct), C.byref(need)))
    ws = torch.empty(max(need.value, 8), dtype=torch.uint8, device=mesh.device)
    _check(lib().hdg_gnn_build_graph(disc.handle, C.byref(mesh.struct), _ptr(H), C.byref(g.struct), _ptr(ws),
                                     C.c_size_t(ws.numel()), _stream(stream)))
    g._ws = ws  # kept until the queued kernels are done with it
    return g


def hdg_gnn_workspace(shape, mesh: Mesh, nprobe=0):
    need = C.c_size_t()
    _check(lib().hdg_gnn_workspace_size(C.byref(_shape(shape)), C.byref(mesh.struct), C.c_int(nprobe),
                                        C.byref(need)))
    return torch.empty(max(need.value, 8), dtype=torch.uint8, device=mesh.device)


def _fb(shp):
    return shp.d2 * (shp.d2 + 1) // 2


def hdg_gnn_forward(shape, params, mesh: Mesh, graph: GnnGraph, N=None, B=None, ws=None, stream=None):
    """Returns (N, B): the lower-block factor entries and every face's block-scaling beta."""
    shp = _shape(shape)
    if N is None:
        N = torch.empty((mesh.nnzb, shp.d2, shp.d2), dtype=torch.float32, device=mesh.device)
    if B is None:
        B = torch.empty((mesh.nfc, _fb(shp)), dtype=torch.float32, device=mesh.device)
    if ws is None:
        ws = hdg_gnn_workspace(shp, mesh, 0)
    _check(lib().hdg_gnn_forward(C.byref(shp), _ptr(params), C.byref(mesh.struct), C.byref(graph.struct), _ptr(N),
                                 _ptr(B), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream)))
    return N, B


def hdg_gnn_loss_grad(shape, params, mesh: Mesh, graph: GnnGraph, probes, N=None, B=None, grad=None, want_grad=True,
                      ws=None, stream=None):
    """Returns (loss as a 1-element device tensor, grad, N, B)."""
    shp = _shape(shape)
    np_ = probes.shape[0]
    if N is None:
        N = torch.empty((mesh.nnzb, shp.d2, shp.d2), dtype=torch.float32, device=mesh.device)
    if B is None:
        B = torch.empty((mesh.nfc, _fb(shp)), dtype=torch.float32, device=mesh.device)
    if want_grad and grad is None:
        grad = torch.empty(hdg_gnn_param_count(shp), dtype=torch.float32, device=mesh.device)
    if ws is None:
        ws = hdg_gnn_workspace(shp, mesh, np_)
    loss = torch.empty(1, dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_gnn_loss_grad(C.byref(shp), _ptr(params), C.byref(mesh.struct), C.byref(graph.struct),
                                   _ptr(probes), C.c_int(np_), _ptr(N), _ptr(B), _ptr(loss),
                                   _ptr(grad) if want_grad else None, _ptr(ws), C.c_size_t(ws.numel()),
                                   _stream(stream)))
    return loss, grad, N, B


def hdg_gnn_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().hdg_gnn_adam(C.c_int64(params.numel()), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), C.c_int(step),
                              C.c_float(lr), C.c_float(beta1), C.c_float(beta2), C.c_float(eps), _stream(stream)))


# ----------------------------------------------------------------------------- FP32 factors + FP64 refinement
def hdg_ir_store_len(disc: Disc) -> int:
    n = C.c_int64()
    _check(lib().hdg_ir_store_len(disc.handle, C.byref(n)))
    return n.value


def hdg_assemble_condense_ir(disc: Disc, mesh: Mesh, kappa, c, f, tau, H, F, X=None, max_sweeps=6, sweeps=None,
                             stream=None):
    _check(lib().hdg_assemble_condense_ir(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(tau),
                                          _ptr(H), _ptr(F), _ptr(X), C.c_int(max_sweeps), _ptr(sweeps),
                                          _stream(stream)))


def hdg_recover_ir(disc: Disc, mesh: Mesh, X, uhat, q=None, u=None, stream=None):
    if q is None:
        q = torch.empty((mesh.nelt, 3, disc.d3), dtype=torch.float64, device=mesh.device)
    if u is None:
        u = torch.empty((mesh.nelt, disc.d3), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_recover_ir(disc.handle, C.byref(mesh.struct), _ptr(X), _ptr(uhat), _ptr(q), _ptr(u),
                                _stream(stream)))
    return q, u


def hdg_export_local_ir(disc: Disc, mesh: Mesh, kappa, c, f, tau, elems, max_sweeps=6, want_x=False, stream=None):
    elems = _dev(elems, torch.int32, mesh.device)
    n = elems.numel()
    m = disc.m
    Cm = torch.empty((n, m, m), dtype=torch.float64, device=mesh.device)
    Cf = torch.empty((n, m), dtype=torch.float64, device=mesh.device)
    X = torch.empty((n, hdg_ir_store_len(disc)), dtype=torch.float64, device=mesh.device) if want_x else None
    _check(lib().hdg_export_local_ir(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f), _ptr(tau),
                                     _ptr(elems), C.c_int64(n), _ptr(Cm), _ptr(Cf), _ptr(X), C.c_int(max_sweeps),
                                     _stream(stream)))
    return Cm, Cf, X



# ----------------------------------------------------------------------------- convection-diffusion
def hdg_elem_face_qp_coords(disc: Disc, mesh: Mesh, out=None, stream=None):
    """Points phi_l^K(qhat_r) of every element's own parametrisation of its faces: [nelt][4][nqd2][3]."""
    if out is None:
        out = torch.empty((mesh.nelt, 4, disc.nqd2, 3), dtype=torch.float64, device=mesh.device)
    _check(lib().hdg_elem_face_qp_coords(disc.handle, C.byref(mesh.struct), _ptr(out), _stream(stream)))
    return out


def hdg_assemble_condense_cd(disc: Disc, mesh: Mesh, kappa, c, f, beta_vol, beta_face, tau, H, F, X=None,
                             stream=None):
    _check(lib().hdg_assemble_condense_cd(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f),
                                          _ptr(beta_vol), _ptr(beta_face), _ptr(tau), _ptr(H), _ptr(F), _ptr(X),
                                          _stream(stream)))


def hdg_export_local_cd(disc: Disc, mesh: Mesh, kappa, c, f, beta_vol, beta_face, tau, elems, want_x=False,
                        stream=None):
    elems = _dev(elems, torch.int32, mesh.device)
    n = elems.numel()
    m = disc.m
    Cm = torch.empty((n, m, m), dtype=torch.float64, device=mesh.device)
    Cf = torch.empty((n, m), dtype=torch.float64, device=mesh.device)
    X = torch.empty((n, hdg_ir_store_len(disc)), dtype=torch.float64, device=mesh.device) if want_x else None
    _check(lib().hdg_export_local_cd(disc.handle, C.byref(mesh.struct), _ptr(kappa), _ptr(c), _ptr(f),
                                     _ptr(beta_vol), _ptr(beta_face), _ptr(tau), _ptr(elems), C.c_int64(n), _ptr(Cm),
                                     _ptr(Cf), _ptr(X), _stream(stream)))
    return Cm, Cf, X


def hdg_solve_gmres_workspace_size(disc: Disc, mesh: Mesh, restart: int) -> int:
    n = C.c_size_t()
    _check(lib().hdg_solve_gmres_workspace_size(disc.handle, C.byref(mesh.struct), C.c_int(restart), C.byref(n)))
    return n.value


def hdg_solve_gmres(disc: Disc, mesh: Mesh, H, b, uhat, rtol=1e-10, max_iter=20000, restart=40, ws=None,
                    stream=None, raise_on_fail=True):
    need = hdg_solve_gmres_workspace_size(disc, mesh, restart)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 8), dtype=torch.uint8, device=mesh.device)
    info = hdg_solve_info()
    code = lib().hdg_solve_gmres(disc.handle, C.byref(mesh.struct), _ptr(H), _ptr(b), _ptr(uhat), C.c_double(rtol),
                                 C.c_int(max_iter), C.c_int(restart), C.byref(info), _ptr(ws),
                                 C.c_size_t(ws.numel()), _stream(stream))
    out = {"iterations": info.iterations, "cycles": info.outer, "rel_residual": info.rel_residual, "status": code,
           "reorthogonalised": info.fell_back}
    if code != 0 and raise_on_fail:
        _check(code)
    return out


# ----------------------------------------------------------------------------- checkpoints
def hdg_gnn_save(path, shape, params, meta=None):
    """params: FP32 vector (any device; copied to the host); meta: {str: str}."""
    shp = _shape(shape)
    h = params.detach().to("cpu", torch.float32).contiguous()
    meta = meta or {}
    keys = (C.c_char_p * max(len(meta), 1))(*[k.encode() for k in meta])
    vals = (C.c_char_p * max(len(meta), 1))(*[str(v).encode() for v in meta.values()])
    _check(lib().hdg_gnn_save(str(path).encode(), C.byref(shp), C.c_void_p(h.data_ptr()), C.c_int64(h.numel()),
                              keys, vals, C.c_int(len(meta))))


def hdg_gnn_load(path):
    """Returns ((d2, hidden, layers), FP32 host tensor of the parameters)."""
    shp = hdg_gnn_shape()
    n = C.c_int64()
    _check(lib().hdg_gnn_load_info(str(path).encode(), C.byref(shp), C.byref(n)))
    h = torch.empty(n.value, dtype=torch.float32)
    _check(lib().hdg_gnn_load(str(path).encode(), C.c_void_p(h.data_ptr()), n))
    return (shp.d2, shp.hidden, shp.layers), h


def hdg_gnn_checkpoint_meta(path, key):
    ln = C.c_size_t()
    _check(lib().hdg_gnn_checkpoint_meta(str(path).encode(), key.encode(), None, C.c_size_t(0), C.byref(ln)))
    buf = C.create_string_buffer(ln.value + 1)
    _check(lib().hdg_gnn_checkpoint_meta(str(path).encode(), key.encode(), buf, C.c_size_t(ln.value + 1),
                                         C.byref(ln)))
    return buf.value.decode()


def hdg_solve_bicgstab(disc: Disc, mesh: Mesh, H, b, uhat, rtol=1e-10, max_iter=20000, check_every=10, ws=None,
                       stream=None, raise_on_fail=True):
    need = C.c_size_t()
    _check(lib().hdg_solve_bicgstab_workspace_size(disc.handle, C.byref(mesh.struct), C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(need.value, 8), dtype=torch.uint8, device=mesh.device)
    info = hdg_solve_info()
    code = lib().hdg_solve_bicgstab(disc.handle, C.byref(mesh.struct), _ptr(H), _ptr(b), _ptr(uhat),
                                    C.c_double(rtol), C.c_int(max_iter), C.c_int(check_every), C.byref(info),
                                    _ptr(ws), C.c_size_t(ws.numel()), _stream(stream))
    out = {"iterations": info.iterations, "restarts": info.outer, "rel_residual": info.rel_residual, "status": code}
    if code != 0 and raise_on_fail:
        _check(code)
    return out
