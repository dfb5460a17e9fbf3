"""Python binding of libpic.so, the MI355X space-charge PIC library (C ABI in include/pic.h).

Argument marshalling only: every step runs in the library's HIP kernels.  PyTorch supplies
device memory (tensors) and the stream (torch's current stream).  Importing this package
raises if the built library is missing; there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpic.so is not built; run `python paper_2208_02382_amd/build.py` "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EHIP, PIC_EDOMAIN, PIC_EUNSUPPORTED, PIC_ENODEV = (
    0, -1, -2, -3, -4, -5, -6)
PIC_EINTERNAL = -7
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EHIP",
                -4: "PIC_EDOMAIN", -5: "PIC_EUNSUPPORTED", -6: "PIC_ENODEV", -7: "PIC_EINTERNAL"}
PUSH_DRIFT, PUSH_THINQUAD, PUSH_KICK = 0, 1, 2
STAGES = ("prologue", "geometry", "green", "deposit", "solve", "gkd", "bin", "unpermute")


class BeamDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("qm_qeeV", ctypes.c_double),
                ("charge_C", ctypes.c_double), ("kin_energy_MeV", ctypes.c_double),
                ("mass_MeV", ctypes.c_double), ("shape", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("grid_fp32", ctypes.c_int), ("space_charge", ctypes.c_int),
                ("tile", ctypes.c_int * 3), ("chunk", ctypes.c_int), ("blocks", ctypes.c_int),
                ("threads", ctypes.c_int), ("direct_field", ctypes.c_int),
                ("deposit_threads", ctypes.c_int)]


ELEM_THIN, ELEM_DRIFT, ELEM_QUAD = 0, 1, 2


class Element(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("ds", ctypes.c_double), ("kind", ctypes.c_int),
                ("nslice", ctypes.c_int)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_SIGS = {
    "pic_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(BeamDesc)]),
    "pic_beam_create": (_I, [ctypes.POINTER(BeamDesc), _P, _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(_P)]),
    "pic_beam_destroy": (_I, [_P]),
    "pic_init_beam": (_I, [_P, ctypes.POINTER(_D), ctypes.c_uint64, _D, _P]),
    "pic_init_beam_from_normals": (_I, [_P, ctypes.POINTER(_D), _P, _P]),
    "pic_init_beam_waterbag": (_I, [_P, ctypes.POINTER(_D), ctypes.c_uint64, _P]),
    "pic_sigma_from_params": (_I, [ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "pic_deposit": (_I, [_P, _P, _P]),
    "pic_poisson_solve": (_I, [_P, _P, _P, _P, _P]),
    "pic_gather": (_I, [_P, _P, _P, _P]),
    "pic_push": (_I, [_P, _I, _D, _P, _P]),
    "pic_track_n_steps": (_I, [_P, ctypes.POINTER(Element), _I, _I, _P]),
    "pic_track_n_steps_diag": (_I, [_P, ctypes.POINTER(Element), _I, _I, _P, _P]),
    "pic_track_n_steps_binned": (_I, [_P, ctypes.POINTER(Element), _I, _I, _P, _P]),
    "pic_moments": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    "pic_objective": (_I, [_P, ctypes.POINTER(_D), _P]),
    "pic_moments_noalloc": (_I, [_P, ctypes.c_int64, _P, _P]),
    "pic_get_geometry": (_I, [_P, ctypes.POINTER(_D), _P]),
    "pic_check": (_I, [_P, _P]),
    "pic_profile_start": (_I, [_P]),
    "pic_profile_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int64)]),
    "pic_adjoint_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(BeamDesc), _I, _I]),
    "pic_track_adjoint": (_I, [_P, ctypes.POINTER(Element), _I, _I, _I, ctypes.POINTER(_D), _P,
                               ctypes.c_size_t, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D),
                               ctypes.POINTER(_D), _P]),
    "pic_batch_workspace_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(ctypes.POINTER(Element)),
                                                     ctypes.POINTER(_I)]),
    "pic_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(ctypes.POINTER(Element)),
                              ctypes.POINTER(_I), _I, _P, ctypes.c_size_t, _P,
                              ctypes.POINTER(_P)]),
    "pic_track_batch": (_I, [_P, _I, _P]),
    "pic_batch_destroy": (_I, [_P]),
    "pic_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class PicError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.pic_last_error().decode()
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))


def _check(status, where):
    if status != PIC_OK:
        raise PicError(status, where)


def last_error():
    return _lib.pic_last_error().decode()


def moments_noalloc(X, out=None):
    """pic_moments_noalloc: the 27 moments (6 means, then the 21 centred second moments, upper
    triangle row-major) of a float64 phase-space tensor X of shape (6, n) on the device, into
    `out` (a float64 device tensor of 27 entries, allocated here if not given), with no
    workspace; enqueued on torch's current stream."""
    assert X.dtype == torch.float64 and X.is_contiguous() and X.dim() == 2 and X.shape[0] == 6
    if out is None:
        out = torch.empty(27, dtype=torch.float64, device=X.device)
    assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 27
    _check(_lib.pic_moments_noalloc(_ptr(X), int(X.shape[1]), _ptr(out), _stream()),
           "pic_moments_noalloc")
    return out


def make_desc(n, qm_qeeV, charge_C, kin_energy_MeV, mass_MeV, shape, nodes, grid_fp32=False,
              space_charge=True, tuning=None, direct_field=False):
    """tuning: None or a dict with any of tile (3 ints), chunk, blocks, threads, deposit_threads
    (0 = default).  direct_field: E' from the field's own integrated Green's functions (no
    differencing)."""
    nx, ny, nz = nodes
    t = tuning or {}
    tile = t.get("tile", (0, 0, 0))
    return BeamDesc(int(n), float(qm_qeeV), float(charge_C), float(kin_energy_MeV),
                    float(mass_MeV), int(shape), int(nx), int(ny), int(nz), int(bool(grid_fp32)),
                    int(bool(space_charge)), (ctypes.c_int * 3)(*[int(v) for v in tile]),
                    int(t.get("chunk", 0)), int(t.get("blocks", 0)), int(t.get("threads", 0)),
                    int(bool(direct_field)), int(t.get("deposit_threads", 0)))


def sigma_from_params(sigmaX, sigmaY, sigmaT, sigmaPx, sigmaPy, sigmaPt, muxpx=0.0, muypy=0.0,
                      mutpt=0.0):
    """6x6 covariance (nested lists) from Listing 1's distribution parameters."""
    p = (ctypes.c_double * 9)(sigmaX, sigmaY, sigmaT, sigmaPx, sigmaPy, sigmaPt, muxpx, muypy,
                              mutpt)
    out = (ctypes.c_double * 36)()
    _check(_lib.pic_sigma_from_params(p, out), "pic_sigma_from_params")
    return [list(out[r * 6:(r + 1) * 6]) for r in range(6)]


def workspace_bytes(desc):
    return int(_lib.pic_workspace_bytes(ctypes.byref(desc)))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _sigma(sigma):
    s = torch.as_tensor(sigma, dtype=torch.float64).reshape(36).tolist()
    return (ctypes.c_double * 36)(*s)


class Beam:
    """A beam bound to device memory owned by torch tensors.

    X is a (6, n) float64 tensor (rows x, px, y, py, z, delta); the workspace is a uint8
    tensor of pic_workspace_bytes.  Grids are float64, or float32 when grid_fp32.
    """

    def __init__(self, n, qm_qeeV, charge_C, kin_energy_MeV, mass_MeV, shape, nodes,
                 grid_fp32=False, space_charge=True, device="cuda:0", X=None, tuning=None,
                 direct_field=False):
        self.desc = make_desc(n, qm_qeeV, charge_C, kin_energy_MeV, mass_MeV, shape, nodes,
                              grid_fp32, space_charge, tuning, direct_field)
        self.device = torch.device(device)
        self.n = int(n)
        self.nodes = tuple(int(v) for v in nodes)
        self.grid_dtype = torch.float32 if grid_fp32 else torch.float64
        nbytes = workspace_bytes(self.desc)
        if nbytes == 0:
            raise PicError(PIC_EINVAL if last_error() else PIC_EUNSUPPORTED, "workspace_bytes")
        if X is None:
            X = torch.empty((6, self.n), dtype=torch.float64, device=self.device)
        assert X.dtype == torch.float64 and X.is_contiguous() and tuple(X.shape) == (6, self.n)
        self.X = X
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.pic_beam_create(ctypes.byref(self.desc), _ptr(self.X), _ptr(self.work),
                                        nbytes, _stream(), ctypes.byref(h)), "pic_beam_create")
        self._h = h

    @classmethod
    def from_config(cls, cfg, grid_fp32=False, space_charge=True, device="cuda:0", n=None,
                    tuning=None):
        """Build from a workloads.Beam-like object (n, qm_qeeV, charge_C, kin_energy_MeV,
        mass_MeV, shape, nodes)."""
        return cls(cfg.n if n is None else n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV,
                   cfg.mass_MeV, cfg.shape, cfg.nodes, grid_fp32, space_charge, device,
                   tuning=tuning)

    def close(self):
        if getattr(self, "_h", None):
            _lib.pic_beam_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- grid allocation helpers
    def new_rho(self):
        nx, ny, nz = self.nodes
        return torch.empty((nz, ny, nx), dtype=self.grid_dtype, device=self.device)

    def new_phi(self):
        nx, ny, nz = self.nodes
        return torch.empty((nz + 2, ny + 2, nx + 2), dtype=self.grid_dtype, device=self.device)

    def new_E(self):
        nx, ny, nz = self.nodes
        return torch.empty((3, nz, ny, nx), dtype=self.grid_dtype, device=self.device)

    def new_Ep(self):
        return torch.empty((3, self.n), dtype=self.grid_dtype, device=self.device)

    # --------------------------------------------------------------- calls of the C ABI
    def init(self, sigma, seed, halo_frac=0.0):
        _check(_lib.pic_init_beam(self._h, _sigma(sigma), int(seed), float(halo_frac),
                                  _stream()), "pic_init_beam")

    def init_waterbag(self, sigma, seed):
        """Uniform inside the 6-D ellipsoid x^T sigma^-1 x <= 8 (covariance sigma)."""
        _check(_lib.pic_init_beam_waterbag(self._h, _sigma(sigma), int(seed), _stream()),
               "pic_init_beam_waterbag")

    def init_from_normals(self, sigma, xi):
        assert xi.dtype == torch.float64 and xi.is_contiguous() and tuple(xi.shape) == (6, self.n)
        _check(_lib.pic_init_beam_from_normals(self._h, _sigma(sigma), _ptr(xi), _stream()),
               "pic_init_beam_from_normals")

    def deposit(self, rho=None):
        rho = self.new_rho() if rho is None else rho
        _check(_lib.pic_deposit(self._h, _ptr(rho), _stream()), "pic_deposit")
        return rho

    def poisson_solve(self, rho, phi=None, E=None):
        E = self.new_E() if E is None else E
        _check(_lib.pic_poisson_solve(self._h, _ptr(rho), _ptr(phi), _ptr(E), _stream()),
               "pic_poisson_solve")
        return phi, E

    def gather(self, E, Ep=None):
        Ep = self.new_Ep() if Ep is None else Ep
        _check(_lib.pic_gather(self._h, _ptr(E), _ptr(Ep), _stream()), "pic_gather")
        return Ep

    def push(self, kind, value, Ep=None):
        _check(_lib.pic_push(self._h, int(kind), float(value), _ptr(Ep), _stream()), "pic_push")

    def track(self, lattice, n_steps, diagnostics=False, binned=False, ids=None):
        """lattice: (k, ds) thin steps or (kind, k, ds, nslice) elements, cycled over the steps.
        diagnostics: also return the moments at the end of every step, a float64 tensor
        (n_steps, 27) on the device (6 means, then the 21 centred second moments, upper
        triangle row-major).  binned: leave X in the library's tile order
        (pic_track_n_steps_binned); ids: optional int32/uint32 labels on the device, n entries,
        permuted with the particles."""
        arr = _lattice(lattice)
        if binned:
            assert not diagnostics
            if ids is not None:
                assert ids.dtype in (torch.int32, torch.uint32) and ids.is_contiguous()
                assert ids.numel() == self.n
            _check(_lib.pic_track_n_steps_binned(self._h, arr, len(lattice), int(n_steps),
                                                 _ptr(ids), _stream()),
                   "pic_track_n_steps_binned")
            return None
        if not diagnostics:
            _check(_lib.pic_track_n_steps(self._h, arr, len(lattice), int(n_steps), _stream()),
                   "pic_track_n_steps")
            return None
        diag = torch.empty((max(int(n_steps), 1), 27), dtype=torch.float64, device=self.device)
        _check(_lib.pic_track_n_steps_diag(self._h, arr, len(lattice), int(n_steps), _ptr(diag),
                                           _stream()), "pic_track_n_steps_diag")
        return diag[:int(n_steps)]

    def moments(self):
        mean = (ctypes.c_double * 6)()
        cov = (ctypes.c_double * 36)()
        _check(_lib.pic_moments(self._h, mean, cov, _stream()), "pic_moments")
        return list(mean), [list(cov[r * 6:(r + 1) * 6]) for r in range(6)]

    def objective(self):
        """(sigma_x, sigma_y, eps_x, eps_y) of the current X, computed by the library."""
        m = (ctypes.c_double * 4)()
        _check(_lib.pic_objective(self._h, m, _stream()), "pic_objective")
        return list(m)

    def geometry(self):
        out = (ctypes.c_double * 9)()
        _check(_lib.pic_get_geometry(self._h, out, _stream()), "pic_get_geometry")
        return list(out[0:3]), list(out[3:6]), list(out[6:9])

    def track_adjoint(self, lattice, n_steps, w, ckpt_every=10, xi=None):
        """Reverse sweep from the current X (= X0): returns (m, dJ/dk, dJ/dX0, dJ/dL or None)
        for J = w . (sigma_x, sigma_y, eps_x, eps_y); X holds the final state afterwards."""
        n_el = len(lattice)
        arr = _lattice(lattice)
        nbytes = int(_lib.pic_adjoint_workspace_bytes(ctypes.byref(self.desc), int(n_steps),
                                                      int(ckpt_every)))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "pic_adjoint_workspace_bytes")
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        lam = torch.empty((6, self.n), dtype=torch.float64, device=self.device)
        wv = (ctypes.c_double * 4)(*[float(v) for v in w])
        m = (ctypes.c_double * 4)()
        dk = (ctypes.c_double * n_el)()
        dL = (ctypes.c_double * 36)()
        if xi is not None:
            assert xi.dtype == torch.float64 and xi.is_contiguous() and tuple(xi.shape) == (6, self.n)
        _check(_lib.pic_track_adjoint(self._h, arr, n_el, int(n_steps), int(ckpt_every), wv,
                                      _ptr(work), nbytes, _ptr(lam), _ptr(xi), m, dk,
                                      dL if xi is not None else None, _stream()),
               "pic_track_adjoint")
        dLm = [list(dL[r * 6:(r + 1) * 6]) for r in range(6)] if xi is not None else None
        return list(m), list(dk), lam, dLm

    def profile_start(self):
        _check(_lib.pic_profile_start(self._h), "pic_profile_start")

    def profile_read(self):
        """{stage: (total ms, launches)} since profile_start; synchronises."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        _check(_lib.pic_profile_read(self._h, ms, cnt), "pic_profile_read")
        return {STAGES[q]: (ms[q], cnt[q]) for q in range(8)}

    def check(self):
        return _lib.pic_check(self._h, _stream())


def _element(e):
    """(k, ds): a thin-lens step; (kind, k, ds, nslice): ELEM_THIN / ELEM_DRIFT / ELEM_QUAD."""
    if len(e) == 2:
        return Element(float(e[0]), float(e[1]), ELEM_THIN, 1)
    kind, k, ds, ns = e
    return Element(float(k), float(ds), int(kind), int(ns))


def _lattice(lattice):
    return (Element * len(lattice))(*[_element(e) for e in lattice])


class Batch:
    """Independent beams tracked together: one launch per stage for all of them, the whole
    step loop replayed from one HIP graph (captured on the first track() with a given step
    count).  The beams share shape and grid precision; particle counts and grids may differ.
    Runs on a stream of its own, ordered after and before torch's current stream."""

    def __init__(self, beams, lattices, blocks_per_beam=0):
        if len(beams) != len(lattices) or not beams:
            raise ValueError("one lattice per beam, at least one beam")
        self.beams = list(beams)
        self.device = self.beams[0].device
        nb = len(self.beams)
        self._lats = [_lattice(l) for l in lattices]
        n_el = (_I * nb)(*[len(l) for l in lattices])
        ptrs = (ctypes.POINTER(Element) * nb)(
            *[ctypes.cast(a, ctypes.POINTER(Element)) for a in self._lats])
        nbytes = int(_lib.pic_batch_workspace_bytes(nb, ptrs, n_el))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "pic_batch_workspace_bytes")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device)
        handles = (_P * nb)(*[b._h for b in self.beams])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            _check(_lib.pic_batch_create(handles, nb, ptrs, n_el, int(blocks_per_beam),
                                         _ptr(self.work), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)), "pic_batch_create")
        self._h = h

    def track(self, n_steps):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(_lib.pic_track_batch(self._h, int(n_steps), ctypes.c_void_p(self.stream.cuda_stream)),
               "pic_track_batch")
        cur.wait_stream(self.stream)

    def check(self):
        """Per-beam device status (pic_check), in beam order."""
        return [b.check() for b in self.beams]

    def close(self):
        if getattr(self, "_h", None):
            _lib.pic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
