"""Python binding of libgrmhd.so (C ABI in include/grmhd.h).

Argument marshalling only: every step of the update runs in the HIP library.  PyTorch
provides device memory and the stream.  Importing this module does not load the
library; the first call does, and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.environ.get("GRMHD_SO", os.path.join(_HERE, "libgrmhd.so"))
_lib = None

ABI_VERSION = 4
OK, EINVAL, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MINK_CART, KS_LOGSPH = 0, 1
PLM_MC, PPM, PLM_MINMOD, PPM_FLAT = 0, 1, 2, 3
LLF, HLLE = 0, 1
BC_OUTFLOW, BC_POLAR, BC_PERIODIC = 0, 1, 2
GUESS_PLAIN, GUESS_MLP = 0, 1
EMF_AVERAGE, EMF_UPWIND = 0, 1
FLOOR_FIXED, FLOOR_DRIFT = 0, 1
REGRID_PRIMITIVE, REGRID_CONSERVED = 0, 1

# every symbol declared in include/grmhd.h
EXPORTS = ("grmhd_sizes", "grmhd_block_layout", "grmhd_init_grid", "grmhd_step",
           "grmhd_cons2prim", "grmhd_divb", "grmhd_plan_dump", "grmhd_geometry_point",
           "grmhd_mlp_sizes", "grmhd_mlp_train_step", "grmhd_mlp_gradients", "grmhd_mlp_pack",
           "grmhd_mlp_forward", "grmhd_prim2cons_batch", "grmhd_mlp_dataset",
           "grmhd_mlp_normalize", "grmhd_extract_cells", "grmhd_destroy", "grmhd_last_error",
           "grmhd_autotune", "grmhd_set_variants", "grmhd_mlp_train_step_noalloc",
           "grmhd_regrid", "grmhd_block_dt")


class BlockDesc(C.Structure):
    _fields_ = [("lev", C.c_int32 * 3), ("lat", C.c_int32), ("org", C.c_int64 * 3),
                ("n", C.c_int32 * 3)]


class GridDesc(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("coords", C.c_int32), ("spin_a", C.c_double),
                ("gamma_ad", C.c_double), ("xmin", C.c_double * 3), ("xmax", C.c_double * 3),
                ("n_eff", C.c_int32 * 3), ("n_ghost", C.c_int32), ("n_blocks", C.c_int32),
                ("n_lat_levels", C.c_int32), ("blocks", C.POINTER(BlockDesc)),
                ("recon", C.c_int32), ("riemann", C.c_int32), ("bc", C.c_int32 * 6),
                ("courant", C.c_double), ("rho_fl_c", C.c_double), ("rho_fl_p", C.c_double),
                ("u_fl_c", C.c_double), ("u_fl_p", C.c_double), ("bsq_rho_max", C.c_double),
                ("bsq_u_max", C.c_double), ("gamma_max", C.c_double), ("c2p_guess", C.c_int32),
                ("c2p_maxit", C.c_int32), ("c2p_tol", C.c_double), ("mlp_weights", C.c_void_p),
                ("batched", C.c_int32), ("profile", C.c_int32), ("emf", C.c_int32),
                ("floor_frame", C.c_int32)]


KERNEL_CLASSES = ("ghost", "bcell", "flux1", "flux2", "flux3", "emf", "update", "dt")


class Buffers(C.Structure):
    _fields_ = [("prim", C.c_void_p), ("bface", C.c_void_p), ("work", C.c_void_p),
                ("work_bytes", C.c_size_t)]


class StepStats(C.Structure):
    _fields_ = [("real_zone_cycles", C.c_int64), ("lat_eff_zone_cycles", C.c_int64),
                ("amr_lat_eff_zone_cycles", C.c_int64), ("steps_per_level", C.c_int64 * 8),
                ("c2p_iter_hist", C.c_int64 * 64), ("c2p_tier", C.c_int64 * 5),
                ("floor_hits", C.c_int64), ("mlp_guesses", C.c_int64), ("dt_min", C.c_double), ("t_sim", C.c_double),
                ("kernel_ms", C.c_double), ("class_ms", C.c_double * 8),
                ("class_launches", C.c_int64 * 8), ("bad_states", C.c_int64)]


class C2PBatch(C.Structure):
    _fields_ = [("n", C.c_int64), ("U", C.c_void_p), ("geom", C.c_void_p), ("guess", C.c_void_p),
                ("prev", C.c_void_p), ("P", C.c_void_p), ("iters", C.c_void_p),
                ("tier", C.c_void_p), ("gamma_ad", C.c_double), ("tol", C.c_double),
                ("maxit", C.c_int32), ("mlp_weights", C.c_void_p)]


# variants of the flux kernel (minimum waves per SIMD, faces per thread) and of the update
# kernel (minimum waves per SIMD), as built
FLUX_WAVES = (1, 2, 4, 2)
FLUX_FACES = (1, 1, 1, 2)
UPDATE_WAVES = (1, 2)
NVAR_FLUX, NVAR_UPD = len(FLUX_WAVES), len(UPDATE_WAVES)


class GrmhdError(RuntimeError):
    pass


def lib():
    """Load libgrmhd.so; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise GrmhdError(f"{SO_PATH} is not built; run paper_1912_10192_amd.build.build()")
        # torch first: the library then binds to the HIP runtime torch has loaded, so
        # torch's streams and device memory are the library's (loaded the other way round,
        # the process holds two runtimes and the library's calls on torch's streams fail)
        import torch  # noqa: F401

        L = C.CDLL(SO_PATH)
        L.grmhd_sizes.argtypes = [C.POINTER(GridDesc), C.POINTER(C.c_size_t),
                                  C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.grmhd_block_layout.argtypes = [C.POINTER(GridDesc), C.c_int32, C.POINTER(C.c_int64),
                                         C.c_int32 * 3]
        L.grmhd_init_grid.argtypes = [C.POINTER(GridDesc), C.POINTER(Buffers), C.c_void_p,
                                      C.POINTER(C.c_void_p)]
        L.grmhd_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(StepStats)]
        L.grmhd_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.grmhd_set_variants.argtypes = [C.c_void_p, C.c_void_p]
        L.grmhd_cons2prim.argtypes = [C.c_void_p, C.POINTER(C2PBatch), C.c_void_p]
        L.grmhd_divb.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_void_p]
        L.grmhd_plan_dump.argtypes = [C.POINTER(GridDesc), C.c_int32, C.c_void_p,
                                      C.POINTER(C.c_size_t)]
        L.grmhd_geometry_point.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                           C.c_void_p, C.c_void_p]
        vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        L.grmhd_mlp_sizes.argtypes = [i32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t)]
        L.grmhd_mlp_train_step.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, f32, vp, vp, vp]
        L.grmhd_mlp_train_step_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, f32, vp, vp]
        L.grmhd_mlp_gradients.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
        L.grmhd_mlp_pack.argtypes = [vp, vp, vp, vp]
        L.grmhd_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.grmhd_prim2cons_batch.argtypes = [i64, vp, vp, vp, f64, vp, vp]
        L.grmhd_mlp_dataset.argtypes = [i64, vp, vp, vp, f64, vp, vp, vp, vp]
        L.grmhd_mlp_normalize.argtypes = [vp, i64, i32, vp, vp, i32, vp]
        L.grmhd_extract_cells.argtypes = [vp, vp, vp, vp]
        L.grmhd_destroy.argtypes = [C.c_void_p]
        L.grmhd_regrid.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.grmhd_block_dt.argtypes = [C.c_void_p, C.c_void_p]
        L.grmhd_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise GrmhdError(f"libgrmhd error {rc}: {lib().grmhd_last_error().decode()}")


def uniform_blocks(n, block, lats=None):
    """blocks of size `block` tiling an n grid, x1 fastest in the block order; lats (one
    time level per x1 block column) gives local time stepping levels by radius"""
    nb = [n[d] // block[d] for d in range(3)]
    if any(nb[d] * block[d] != n[d] for d in range(3)):
        raise ValueError("block size must divide the grid")
    out = []
    for k in range(nb[2]):
        for j in range(nb[1]):
            for i in range(nb[0]):
                out.append(dict(org=(i * block[0], j * block[1], k * block[2]), n=tuple(block),
                                lev=(0, 0, 0), lat=int(lats[i]) if lats is not None else 0))
    return out


class Desc:
    """Owns a GridDesc and its block array built from a workload dict (configs.py)."""

    def __init__(self, cfg: dict, blocks=None, batched=False, profile=False, mlp_blob=None):
        blocks = blocks if blocks is not None else uniform_blocks(cfg["n"], cfg.get("block", cfg["n"]))
        self.cfg = cfg
        self.blocks = (BlockDesc * len(blocks))()
        for b, bd in enumerate(blocks):
            for d in range(3):
                self.blocks[b].lev[d] = bd["lev"][d]
                self.blocks[b].org[d] = bd["org"][d]
                self.blocks[b].n[d] = bd["n"][d]
            self.blocks[b].lat = bd["lat"]
        d = GridDesc()
        d.abi_version = ABI_VERSION
        d.coords = cfg["coords"]
        d.spin_a = cfg.get("a", 0.0)
        d.gamma_ad = cfg["gam"]
        for k in range(3):
            d.xmin[k] = cfg["xlo"][k]
            d.xmax[k] = cfg["xhi"][k]
            d.n_eff[k] = cfg["n"][k]
        d.n_ghost = cfg["ng"]
        d.n_blocks = len(blocks)
        d.n_lat_levels = max(int(bd["lat"]) for bd in blocks) + 1
        d.blocks = C.cast(self.blocks, C.POINTER(BlockDesc))
        d.recon = cfg["recon"]
        d.riemann = cfg["riemann"]
        for k in range(6):
            d.bc[k] = cfg["bc"][k]
        d.courant = cfg.get("courant", 0.8)
        d.rho_fl_c = cfg.get("rho_fl_c", 0.0)
        d.rho_fl_p = cfg.get("rho_fl_p", 0.0)
        d.u_fl_c = cfg.get("u_fl_c", 0.0)
        d.u_fl_p = cfg.get("u_fl_p", 0.0)
        d.bsq_rho_max = cfg.get("bsq_rho_max", 1e300)
        d.bsq_u_max = cfg.get("bsq_u_max", 1e300)
        d.gamma_max = cfg.get("gamma_max", 1e150)
        d.c2p_guess = GUESS_MLP if mlp_blob is not None else GUESS_PLAIN
        d.c2p_maxit = cfg.get("maxit", 50)
        d.c2p_tol = cfg.get("tol", 1e-12)
        d.mlp_weights = mlp_blob.data_ptr() if mlp_blob is not None else None
        self.mlp_blob = mlp_blob
        d.batched = int(batched) if not isinstance(batched, bool) else (1 if batched else 0)
        d.profile = 1 if profile else 0
        d.emf = int(cfg.get("emf", EMF_AVERAGE))
        d.floor_frame = int(cfg.get("floor_frame", FLOOR_FIXED))
        self.d = d

    def sizes(self):
        p, b, w = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(lib().grmhd_sizes(C.byref(self.d), C.byref(p), C.byref(b), C.byref(w)))
        return p.value, b.value, w.value

    def layout(self, b):
        off = C.c_int64()
        np_ = (C.c_int32 * 3)()
        _check(lib().grmhd_block_layout(C.byref(self.d), b, C.byref(off), np_))
        return off.value, tuple(np_)

    def plan_raw(self, what):
        """raw bytes of a device list (plan_dump 15..19)"""
        nbytes = C.c_size_t()
        _check(lib().grmhd_plan_dump(C.byref(self.d), what, None, C.byref(nbytes)))
        buf = np.zeros(nbytes.value, dtype=np.uint8)
        _check(lib().grmhd_plan_dump(C.byref(self.d), what, buf.ctypes.data_as(C.c_void_p),
                                     C.byref(nbytes)))
        return buf

    def plan_dump(self, what):
        nbytes = C.c_size_t()
        _check(lib().grmhd_plan_dump(C.byref(self.d), what, None, C.byref(nbytes)))
        buf = np.zeros(nbytes.value // 4, dtype=np.int32)
        _check(lib().grmhd_plan_dump(C.byref(self.d), what, buf.ctypes.data_as(C.c_void_p),
                                     C.byref(nbytes)))
        return buf.reshape(-1, {9: 13, 12: 10, 13: 7, 14: 7, 20: 6}.get(what, 4))


def geometry_point(coords, a, x1, x2):
    out = np.zeros(15)
    conn = np.zeros(40)
    _check(lib().grmhd_geometry_point(coords, a, x1, x2, out.ctypes.data_as(C.c_void_p),
                                      conn.ctypes.data_as(C.c_void_p)))
    return out, conn


# ------------------------------------------------------------------ state layout

def scatter(desc: Desc, P, B1, B2, B3):
    """global interior arrays -> packed per-block host arrays (prim, bface)"""
    g = desc.cfg["ng"]
    nprim, nbface, _ = desc.sizes()
    prim = np.zeros(nprim)
    bface = np.zeros(nbface)
    for b in range(desc.d.n_blocks):
        off, (n1p, n2p, n3p) = desc.layout(b)
        V = n1p * n2p * n3p
        bd = desc.blocks[b]
        o = [bd.org[d] for d in range(3)]
        n = [bd.n[d] for d in range(3)]
        pv = prim[5 * off:5 * off + 5 * V].reshape(5, n3p, n2p, n1p)
        bv = bface[3 * off:3 * off + 3 * V].reshape(3, n3p, n2p, n1p)
        pv[:, g:g + n[2], g:g + n[1], g:g + n[0]] = P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1],
                                                     o[0]:o[0] + n[0]]
        bv[0, g:g + n[2], g:g + n[1], g:g + n[0] + 1] = B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1],
                                                          o[0]:o[0] + n[0] + 1]
        bv[1, g:g + n[2], g:g + n[1] + 1, g:g + n[0]] = B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1,
                                                          o[0]:o[0] + n[0]]
        bv[2, g:g + n[2] + 1, g:g + n[1], g:g + n[0]] = B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1],
                                                          o[0]:o[0] + n[0]]
    return prim, bface


def gather(desc: Desc, prim, bface):
    """packed per-block host arrays -> global interior arrays (P, B1, B2, B3)"""
    g = desc.cfg["ng"]
    N1, N2, N3 = desc.cfg["n"]
    P = np.zeros((5, N3, N2, N1))
    B1 = np.zeros((N3, N2, N1 + 1))
    B2 = np.zeros((N3, N2 + 1, N1))
    B3 = np.zeros((N3 + 1, N2, N1))
    for b in range(desc.d.n_blocks):
        off, (n1p, n2p, n3p) = desc.layout(b)
        V = n1p * n2p * n3p
        bd = desc.blocks[b]
        o = [bd.org[d] for d in range(3)]
        n = [bd.n[d] for d in range(3)]
        pv = prim[5 * off:5 * off + 5 * V].reshape(5, n3p, n2p, n1p)
        bv = bface[3 * off:3 * off + 3 * V].reshape(3, n3p, n2p, n1p)
        P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]] = pv[:, g:g + n[2], g:g + n[1],
                                                                        g:g + n[0]]
        B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0] + 1] = bv[0, g:g + n[2], g:g + n[1],
                                                                          g:g + n[0] + 1]
        B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1, o[0]:o[0] + n[0]] = bv[1, g:g + n[2],
                                                                          g:g + n[1] + 1, g:g + n[0]]
        B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1], o[0]:o[0] + n[0]] = bv[2, g:g + n[2] + 1,
                                                                          g:g + n[1], g:g + n[0]]
    return P, B1, B2, B3


def _block_views(desc: Desc, prim, bface, b):
    off, (n1p, n2p, n3p) = desc.layout(b)
    V = n1p * n2p * n3p
    return (prim[5 * off:5 * off + 5 * V].reshape(5, n3p, n2p, n1p),
            bface[3 * off:3 * off + 3 * V].reshape(3, n3p, n2p, n1p))


def scatter_blocks(desc: Desc, states):
    """per-block interior arrays (P[5][n3][n2][n1], B1[n3][n2][n1+1], B2[n3][n2+1][n1],
    B3[n3+1][n2][n1]) -> packed host arrays (prim, bface)"""
    g = desc.cfg["ng"]
    nprim, nbface, _ = desc.sizes()
    prim = np.zeros(nprim)
    bface = np.zeros(nbface)
    for b, (P, B1, B2, B3) in enumerate(states):
        n = [desc.blocks[b].n[d] for d in range(3)]
        pv, bv = _block_views(desc, prim, bface, b)
        pv[:, g:g + n[2], g:g + n[1], g:g + n[0]] = P
        bv[0, g:g + n[2], g:g + n[1], g:g + n[0] + 1] = B1
        bv[1, g:g + n[2], g:g + n[1] + 1, g:g + n[0]] = B2
        bv[2, g:g + n[2] + 1, g:g + n[1], g:g + n[0]] = B3
    return prim, bface


def gather_blocks(desc: Desc, prim, bface):
    g = desc.cfg["ng"]
    out = []
    for b in range(desc.d.n_blocks):
        n = [desc.blocks[b].n[d] for d in range(3)]
        pv, bv = _block_views(desc, prim, bface, b)
        out.append((pv[:, g:g + n[2], g:g + n[1], g:g + n[0]].copy(),
                    bv[0, g:g + n[2], g:g + n[1], g:g + n[0] + 1].copy(),
                    bv[1, g:g + n[2], g:g + n[1] + 1, g:g + n[0]].copy(),
                    bv[2, g:g + n[2] + 1, g:g + n[1], g:g + n[0]].copy()))
    return out


# ------------------------------------------------------------------ device grid

class Grid:
    """A grid on the GPU: caller-owned torch buffers plus the library context."""

    def __init__(self, cfg: dict, state=None, blocks=None, batched=False, profile=False,
                 mlp_blob=None, device="cuda", pool=None):
        """pool: (prim, bface, work) device tensors (float64, float64, uint8) to place the
        grid's buffers in, in place of new allocations; each must hold at least what
        grmhd_sizes asks (plus 256 bytes of alignment for work).  The grid's buffers are
        then views of them, zeroed here."""
        import torch

        self.torch = torch
        self.cfg, self.batched, self.mlp_blob = dict(cfg), batched, mlp_blob
        self.desc = Desc(cfg, blocks=blocks, batched=batched, profile=profile, mlp_blob=mlp_blob)
        nprim, nbface, nwork = self.desc.sizes()
        self.device = torch.device(device)
        if pool is None:
            self.prim = torch.zeros(nprim, dtype=torch.float64, device=self.device)
            self.bface = torch.zeros(nbface, dtype=torch.float64, device=self.device)
            self.work = torch.empty(nwork + 256, dtype=torch.uint8, device=self.device)
        else:
            pp, pb, pw = pool
            if pp.numel() < nprim or pb.numel() < nbface or pw.numel() < nwork + 256:
                raise GrmhdError(f"pool buffers ({pp.numel()}, {pb.numel()}, {pw.numel()}) smaller "
                                 f"than the layout needs ({nprim}, {nbface}, {nwork + 256})")
            self.prim, self.bface, self.work = pp[:nprim], pb[:nbface], pw[:nwork + 256]
            self.prim.zero_()
            self.bface.zero_()
        if state is not None:
            self.set_state(*state)
        wp = self.work.data_ptr()
        wp_al = (wp + 255) & ~255
        self.bufs = Buffers(self.prim.data_ptr(), self.bface.data_ptr(), wp_al, nwork)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        _check(lib().grmhd_init_grid(C.byref(self.desc.d), C.byref(self.bufs),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)))

    def close(self):
        if self.ctx:
            lib().grmhd_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, P, B1, B2, B3):
        prim, bface = scatter(self.desc, P, B1, B2, B3)
        self.prim.copy_(self.torch.from_numpy(prim))
        self.bface.copy_(self.torch.from_numpy(bface))

    def get_state(self):
        self.torch.cuda.synchronize(self.device)
        return gather(self.desc, self.prim.cpu().numpy(), self.bface.cpu().numpy())

    def set_blocks(self, states):
        """per-block interior arrays (block grids with refinement levels)"""
        prim, bface = scatter_blocks(self.desc, states)
        self.prim.copy_(self.torch.from_numpy(prim))
        self.bface.copy_(self.torch.from_numpy(bface))

    def get_blocks(self):
        self.torch.cuda.synchronize(self.device)
        return gather_blocks(self.desc, self.prim.cpu().numpy(), self.bface.cpu().numpy())

    def step(self, n=1, stats=True):
        st = StepStats() if stats else None
        _check(lib().grmhd_step(self.ctx, n, C.byref(st) if stats else None))
        return st

    def extract_cells(self):
        """every interior cell as flat batches (P[5][n], B[3][n], geom[15][n]) on the device"""
        torch = self.torch
        n = sum(int(np.prod([bd.n[d] for d in range(3)])) for bd in self.desc.blocks)
        P = torch.empty((5, n), dtype=torch.float64, device=self.device)
        B = torch.empty((3, n), dtype=torch.float64, device=self.device)
        G = torch.empty((15, n), dtype=torch.float64, device=self.device)
        _check(lib().grmhd_extract_cells(self.ctx, P.data_ptr(), B.data_ptr(), G.data_ptr()))
        return P, B, G

    def autotune(self):
        """time the kernel variants on the current state and keep the fastest; returns
        the chosen variants and the milliseconds per variant"""
        nf, nu = NVAR_FLUX, NVAR_UPD
        choice = (C.c_int32 * 5)()
        ms = (C.c_double * (3 * nf + 2 * nu))()
        _check(lib().grmhd_autotune(self.ctx, choice, ms))
        return {"flux": [choice[k] for k in range(3)], "update": choice[3],
                "update_split": choice[4],
                "flux_waves": FLUX_WAVES, "flux_faces": FLUX_FACES, "update_waves": UPDATE_WAVES,
                "flux_ms": [[ms[d * nf + v] for v in range(nf)] for d in range(3)],
                "update_ms": [ms[3 * nf + v] for v in range(nu)],
                "update_split_ms": [ms[3 * nf + nu + v] for v in range(nu)]}

    def set_variants(self, flux=(2, 2, 2), update=0, split=0):
        choice = (C.c_int32 * 5)(flux[0], flux[1], flux[2], update, split)
        _check(lib().grmhd_set_variants(self.ctx, choice))

    def regrid(self, blocks, batched=None, conserved=False, pool=None):
        """a new Grid of the same workload on the block layout `blocks`, filled from this
        grid's state (grmhd_regrid; conserved: restrict and prolong the conserved vector);
        this grid keeps its state.  Where the new layout adds or drops a finest level, its
        effective grid doubles or halves in that dimension."""
        old_l = [max(int(b.lev[d]) for b in self.desc.blocks) for d in range(3)]
        new_l = [max(int(b.get("lev", (0, 0, 0))[d]) for b in blocks) for d in range(3)]
        n = tuple((int(self.cfg["n"][d]) >> old_l[d]) << new_l[d] for d in range(3))
        new = Grid(dict(self.cfg, n=n), blocks=blocks,
                   batched=self.batched if batched is None else batched, mlp_blob=self.mlp_blob,
                   pool=pool)
        _check(lib().grmhd_regrid(self.ctx, new.ctx, REGRID_CONSERVED if conserved else REGRID_PRIMITIVE))
        return new

    def block_dt(self):
        """each block's own Courant step (grmhd_block_dt), as a numpy array"""
        out = np.zeros(len(self.desc.blocks))
        _check(lib().grmhd_block_dt(self.ctx, out.ctypes.data_as(C.c_void_p)))
        return out

    def divb(self):
        a, r = C.c_double(), C.c_double()
        _check(lib().grmhd_divb(self.ctx, C.byref(a), C.byref(r), None))
        return a.value, r.value

    def divb_field(self):
        """(max |div B|, its relative form, the per-cell values as a global interior
        array [n3][n2][n1])"""
        a, r = C.c_double(), C.c_double()
        field = self.torch.zeros_like(self.prim)
        _check(lib().grmhd_divb(self.ctx, C.byref(a), C.byref(r), C.c_void_p(field.data_ptr())))
        self.torch.cuda.synchronize(self.device)
        P, _, _, _ = gather(self.desc, field.cpu().numpy(), np.zeros(self.bface.numel()))
        return a.value, r.value, P[0]


def cons2prim_batch(U, geom, guess, prev, gam, tol=1e-12, maxit=50, mlp_blob=None):
    """flat-batch inversion on the GPU; all inputs float64 CUDA tensors [k][n]; with
    mlp_blob the first guess is the network's (guess may be None)"""
    import torch

    n = U.shape[1]
    P = torch.empty((5, n), dtype=torch.float64, device=U.device)
    iters = torch.empty(n, dtype=torch.int32, device=U.device)
    tier = torch.empty(n, dtype=torch.int32, device=U.device)
    b = C2PBatch(n, U.data_ptr(), geom.data_ptr(), guess.data_ptr() if guess is not None else None,
                 prev.data_ptr(), P.data_ptr(), iters.data_ptr(), tier.data_ptr(), gam, tol, maxit,
                 mlp_blob.data_ptr() if mlp_blob is not None else None)
    stream = torch.cuda.current_stream(U.device)
    _check(lib().grmhd_cons2prim(None, C.byref(b), C.c_void_p(stream.cuda_stream)))
    return P, iters, tier


# ------------------------------------------------------------------ learned guess

def _stream(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_sizes(batch):
    a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(lib().grmhd_mlp_sizes(batch, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def prim2cons_batch(P, B, geom, gam):
    import torch
    n = P.shape[1]
    U = torch.empty((9, n), dtype=torch.float64, device=P.device)
    _check(lib().grmhd_prim2cons_batch(n, P.data_ptr(), B.data_ptr(), geom.data_ptr(), gam,
                                       U.data_ptr(), _stream(P)))
    return U


def mlp_dataset(U, P, geom, gam):
    """raw features X[n][8], raw targets Y[n][2] (or None) and the finite-mask"""
    import torch
    n = U.shape[1]
    X = torch.empty((n, 8), dtype=torch.float32, device=U.device)
    Y = torch.empty((n, 2), dtype=torch.float32, device=U.device) if P is not None else None
    ok = torch.empty(n, dtype=torch.int32, device=U.device)
    _check(lib().grmhd_mlp_dataset(n, U.data_ptr(), P.data_ptr() if P is not None else None,
                                   geom.data_ptr(), gam, X.data_ptr(),
                                   Y.data_ptr() if Y is not None else None, ok.data_ptr(),
                                   _stream(U)))
    return X, Y, ok


def mlp_normalize(A, mean=None, sd=None):
    """normalise columns of A in place; computes mean/sd when they are not given"""
    import torch
    n, cols = A.shape
    compute = mean is None
    if compute:
        mean = torch.empty(cols, dtype=torch.float32, device=A.device)
        sd = torch.empty(cols, dtype=torch.float32, device=A.device)
    _check(lib().grmhd_mlp_normalize(A.data_ptr(), n, cols, mean.data_ptr(), sd.data_ptr(),
                                     1 if compute else 0, _stream(A)))
    return mean, sd


def mlp_pack(params, norm):
    import torch
    _, nblob, _ = mlp_sizes(1)
    blob = torch.zeros(nblob, dtype=torch.uint8, device=params.device)
    _check(lib().grmhd_mlp_pack(params.data_ptr(), norm.data_ptr(), blob.data_ptr(), _stream(params)))
    return blob


def mlp_forward(blob, X):
    import torch
    n = X.shape[0]
    Y = torch.empty((n, 2), dtype=torch.float32, device=X.device)
    _check(lib().grmhd_mlp_forward(blob.data_ptr(), X.data_ptr(), n, Y.data_ptr(), _stream(X)))
    return Y


def mlp_gradients(params, X, Y, idx, work=None):
    import torch
    batch = idx.shape[0]
    nparam, _, nwork = mlp_sizes(batch)
    work = work if work is not None else torch.empty(nwork, dtype=torch.float32, device=X.device)
    grad = torch.empty(nparam, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().grmhd_mlp_gradients(params.data_ptr(), X.data_ptr(), Y.data_ptr(), idx.data_ptr(),
                                     batch, work.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                                     _stream(X)))
    return grad, loss


class MLPTrainer:
    """FP32 master weights + Adam state on the device; every step runs in the library."""

    def __init__(self, params, batch=4096):
        import torch
        self.torch = torch
        self.batch = batch
        self.params = params.clone().contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        _, _, nwork = mlp_sizes(batch)
        self.work = torch.empty(nwork, dtype=torch.float32, device=params.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.t = 0

    def step(self, X, Y, idx, lr):
        self.t += 1
        _check(lib().grmhd_mlp_train_step(self.params.data_ptr(), self.m.data_ptr(),
                                          self.v.data_ptr(), self.t, X.data_ptr(), Y.data_ptr(),
                                          idx.data_ptr(), idx.shape[0], lr, self.work.data_ptr(),
                                          self.loss.data_ptr(), _stream(X)))


NOALLOC_MAX_BATCH = 8192


def mlp_train_step_noalloc(params, m, v, step, X, Y, idx, lr, loss):
    """one Adam step through the allocation-free entry point (scratch in the library's
    static device array); params, m, v updated in place, loss[0] receives the batch loss"""
    _check(lib().grmhd_mlp_train_step_noalloc(params.data_ptr(), m.data_ptr(), v.data_ptr(),
                                              step, X.data_ptr(), Y.data_ptr(), idx.data_ptr(),
                                              idx.shape[0], lr, loss.data_ptr(), _stream(X)))


def lat_levels_by_radius(cfg, edges):
    """time level of each x1 block column from its inner radius: level l for
    edges[l-1] <= r_inner < edges[l] (edges increasing), clipped so neighbours differ by
    at most one level"""
    import math
    nb1 = cfg["n"][0] // cfg["block"][0]
    dx1 = (cfg["xhi"][0] - cfg["xlo"][0]) / cfg["n"][0]
    lats = []
    for i in range(nb1):
        r = math.exp(cfg["xlo"][0] + i * cfg["block"][0] * dx1)
        lats.append(sum(1 for e in edges if r >= e))
    for i in range(1, nb1):
        lats[i] = min(lats[i], lats[i - 1] + 1)
    return lats
