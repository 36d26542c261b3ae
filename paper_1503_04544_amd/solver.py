"""Python front of the ccdvm C-ABI.

PyTorch only provides device memory and the stream: every step of the method
runs in the HIP kernels of libccdvm.so, reached through ctypes.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._capi import CCError, lib, make_body, make_config


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Solver:
    """One flow problem bound to one stream of one GPU."""

    def __init__(self, cfg, device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None,
                 static_scratch: bool = False):
        """static_scratch: bind with cc_bind_noalloc (the library's static
        scratch array instead of a scratch tensor)."""
        self.cfg = cfg
        self.device = torch.device(device)
        self._cfg = make_config(cfg)
        self._body = make_body(cfg.body)
        h = C.c_void_p()
        st = lib().cc_create(C.byref(self._cfg), C.byref(self._body), C.byref(h))
        if st != 0:
            raise CCError(st, "cc_create rejected the configuration")
        self._h = h
        sb, gb, xb = C.c_size_t(), C.c_size_t(), C.c_size_t()
        self._check(lib().cc_workspace_bytes(h, C.byref(sb), C.byref(gb), C.byref(xb)))
        self.dim = cfg.dim
        self.ncell = cfg.n[0] * cfg.n[1] * cfg.n[2]
        # octree mesh (also every 3D body that turns): the cells are the leaves
        self.turning = cfg.dim == 3 and cfg.body.motion != "fixed" and cfg.body.kind != "none"
        self.amr = getattr(cfg, "amr_depth", 0) > 0 or self.turning
        if self.amr:
            self._refresh_counts()
        self.nvel = cfg.nv ** cfg.dim
        with torch.cuda.device(self.device):
            # caller-owned device buffers (uint8 tensors; 256-byte aligned by the caching allocator)
            self.state = [torch.empty(sb.value, dtype=torch.uint8, device=self.device) for _ in range(2)]
            self.geom = torch.empty(gb.value, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if static_scratch:
                self.scratch = None
                self._check(lib().cc_bind_noalloc(h, _ptr(self.state[0]), _ptr(self.state[1]), _ptr(self.geom),
                                                  C.c_void_p(self.stream.cuda_stream)))
            else:
                self.scratch = torch.empty(xb.value, dtype=torch.uint8, device=self.device)
                self._check(lib().cc_bind(h, _ptr(self.state[0]), _ptr(self.state[1]), _ptr(self.geom),
                                          _ptr(self.scratch), C.c_void_p(self.stream.cuda_stream)))

    def _refresh_counts(self):
        nl, nf = C.c_int(), C.c_int()
        self._check(lib().cc_amr_counts(self._h, C.byref(nl), C.byref(nf)))
        self.ncell, self.nface = nl.value, nf.value

    def _check(self, st):
        if st != 0:
            msg = lib().cc_last_error(self._h) if getattr(self, "_h", None) else b""
            raise CCError(st, (msg or b"").decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().cc_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- state
    @property
    def dt(self) -> float:
        d = C.c_double()
        self._check(lib().cc_dt(self._h, C.byref(d)))
        return d.value

    def cfl_number(self) -> list:
        """Positivity number of eq. eq-CFL: [transport part, collision part, sum]."""
        out = (C.c_double * 3)()
        self._check(lib().cc_cfl_number(self._h, out))
        return [float(x) for x in out]

    def init_maxwellian(self):
        self._check(lib().cc_init_maxwellian(self._h))

    def load_state(self, f: torch.Tensor, g: torch.Tensor | None = None):
        f = f.to(self.device, torch.float64).contiguous()
        if g is not None:
            g = g.to(self.device, torch.float64).contiguous()
        assert f.numel() == self.ncell * self.nvel
        self._check(lib().cc_load_state(self._h, _ptr(f), _ptr(g)))
        self.stream.synchronize()

    def store_state(self):
        f = torch.empty((self.ncell, self.nvel), dtype=torch.float64, device=self.device)
        g = torch.empty_like(f) if self.dim == 2 else None
        self._check(lib().cc_store_state(self._h, _ptr(f), _ptr(g)))
        self.stream.synchronize()
        return f, g

    # ---------------------------------------------------------------- stepping
    def step(self, nsteps: int = 1, diag: torch.Tensor | bool | None = None):
        """Advance nsteps; with diag=True returns a (nsteps, 4) device tensor of
        (Fx, Fy, torque, mass) of the state at the start of each step (3D fixed
        body: (Fx, Fy, Fz, mass)).  A turning 3D body adapts the mesh every
        step, so ncell (the leaf count) may change."""
        d = None
        if diag is True:
            d = torch.empty((nsteps, 4), dtype=torch.float64, device=self.device)
        elif isinstance(diag, torch.Tensor):
            d = diag
        self._check(lib().cc_step(self._h, int(nsteps), _ptr(d)))
        if self.turning:
            self._refresh_counts()
        return d

    def moments(self) -> torch.Tensor:
        k = 9 if self.dim == 2 else 14
        out = torch.empty((self.ncell, k), dtype=torch.float64, device=self.device)
        self._check(lib().cc_moments(self._h, _ptr(out)))
        return out

    def body_force(self) -> np.ndarray:
        out = (C.c_double * 4)()
        self._check(lib().cc_body_force(self._h, out))
        return np.array(out[:])

    def body_state(self) -> np.ndarray:
        out = (C.c_double * 6)()
        self._check(lib().cc_body_state(self._h, out))
        return np.array(out[:])

    def rigid_update(self, force, torque: float):
        f = (C.c_double * 3)(*[float(x) for x in force])
        self._check(lib().cc_rigid_update(self._h, f, float(torque)))

    # ---------------------------------------------------------------- geometry
    def geometry(self) -> dict:
        """Geometry tables as host arrays.  3D: 'S' (ncell, 6) gas areas of
        the faces x-, x+, y-, y+, z-, z+; 'sw' wall area; 'nw', 'rw' (ncell, 3)
        wall normal and centre; 'vbar', 'vcv' volumes."""
        n = self.ncell
        out = {"type": np.zeros(n, np.int32), "master": np.zeros(n, np.int32)}
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        if self.dim == 2:
            names = ["lxm", "lxp", "lym", "lyp", "lw", "nwx", "nwy", "rwx", "rwy", "sbar", "scv"]
            for k in names:
                out[k] = np.zeros(n)
            self._check(lib().cc_geometry_export(self._h, P(out["type"]), P(out["master"]),
                                                 *[P(out[k]) for k in names]))
            return out
        names = ["sxm", "sxp", "sym", "syp", "szm", "szp", "aw", "nwx", "nwy", "nwz",
                 "rwx", "rwy", "rwz", "vbar", "vcv"]
        raw = {k: np.zeros(n) for k in names}
        self._check(lib().cc_geometry_export3d(self._h, P(out["type"]), P(out["master"]),
                                               *[P(raw[k]) for k in names]))
        out["S"] = np.stack([raw[k] for k in names[:6]], axis=1)
        out["sw"] = raw["aw"]
        out["nw"] = np.stack([raw["nwx"], raw["nwy"], raw["nwz"]], axis=1)
        out["rw"] = np.stack([raw["rwx"], raw["rwy"], raw["rwz"]], axis=1)
        out["vbar"], out["vcv"] = raw["vbar"], raw["vcv"]
        return out

    def amr_leaves(self) -> dict:
        """Octree leaves (host arrays): depth, coordinates at that depth,
        type, master, gas volume, control-volume volume, wall area, face
        gas areas (n, 6)."""
        n = self.ncell
        out = {"lvl": np.zeros(n, np.int32), "ijk": np.zeros((n, 3), np.int32),
               "type": np.zeros(n, np.int32), "master": np.zeros(n, np.int32),
               "vbar": np.zeros(n), "vcv": np.zeros(n), "sw": np.zeros(n), "S": np.zeros((n, 6))}
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(lib().cc_amr_export(self._h, *[P(out[k]) for k in
                                                   ("lvl", "ijk", "type", "master", "vbar", "vcv", "sw", "S")]))
        return out

    def amr_faces(self) -> dict:
        out = {"ptr": np.zeros(self.ncell + 1, np.int32), "nb": np.zeros(self.nface, np.int32),
               "dir": np.zeros(self.nface, np.int32), "area": np.zeros(self.nface)}
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(lib().cc_amr_faces(self._h, *[P(out[k]) for k in ("ptr", "nb", "dir", "area")]))
        return out

    def counts(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(lib().cc_geometry_counts(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def adjoint(self, nsteps: int, ckpt_every: int = 16, objective: str = "drag", pool=None):
        """J and dJ/d(T_w, Kn, Ma) of the drag or torque after nsteps from the
        inflow Maxwellian (hand-written adjoint with checkpointing).  pool: a
        device uint8 tensor of at least adjoint_workspace_bytes() bytes to
        use, else one is allocated for the call."""
        nb = C.c_size_t()
        self._check(lib().cc_adjoint_workspace_bytes(self._h, int(nsteps), int(ckpt_every), C.byref(nb)))
        if pool is None:
            pool = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        elif pool.numel() < nb.value:
            raise ValueError(f"adjoint pool of {pool.numel()} bytes, {nb.value} needed")
        out = (C.c_double * 4)()
        self._check(lib().cc_adjoint(self._h, int(nsteps), int(ckpt_every),
                                     0 if objective == "drag" else 1, _ptr(pool), out))
        return out[0], np.array(out[1:])

    def adjoint_workspace_bytes(self, nsteps: int, ckpt_every: int = 16) -> int:
        """Bytes of the device pool adjoint() allocates (cc_adjoint_workspace_bytes)."""
        nb = C.c_size_t()
        self._check(lib().cc_adjoint_workspace_bytes(self._h, int(nsteps), int(ckpt_every), C.byref(nb)))
        return nb.value

    def set_tile_rows(self, rows: int):
        self._check(lib().cc_set_tile_rows(self._h, int(rows)))

    # ---------------------------------------------------------------- profiling
    def profile_enable(self, on: bool = True):
        self._check(lib().cc_profile_enable(self._h, int(on)))

    def profile_read(self, kernel: int):
        ms, n = C.c_double(), C.c_int()
        self._check(lib().cc_profile_read(self._h, kernel, C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Batch:
    """Several Solvers on the same stream advanced together (cc_batch_*)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        h = C.c_void_p()
        st = lib().cc_batch_create(arr, len(self.solvers), C.byref(h))
        if st != 0:
            raise CCError(st, "cc_batch_create rejected the instances")
        self._h = h
        nb = C.c_size_t()
        self._check(lib().cc_batch_workspace_bytes(h, C.byref(nb)))
        dev = self.solvers[0].device
        self.workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
        self._check(lib().cc_batch_bind(h, _ptr(self.workspace)))

    def _check(self, st):
        if st != 0:
            msg = lib().cc_batch_last_error(self._h) if getattr(self, "_h", None) else b""
            raise CCError(st, (msg or b"").decode())

    def groups(self):
        n = C.c_int()
        ch = (C.c_int * 16)()
        rows = (C.c_int * 16)()
        self._check(lib().cc_batch_groups(self._h, C.byref(n), ch, rows))
        return [(ch[i], rows[i]) for i in range(n.value)]

    def autotune(self, trial_steps: int = 5):
        n = len(self.groups())
        out = (C.c_int * max(n, 1))()
        self._check(lib().cc_batch_autotune(self._h, int(trial_steps), out))
        return list(out[:n])

    def step(self, nsteps: int = 1):
        self._check(lib().cc_batch_step(self._h, int(nsteps)))

    def adjoint_workspace_bytes(self, nsteps: int, ckpt_every: int = 16) -> int:
        nb = C.c_size_t()
        self._check(lib().cc_batch_adjoint_workspace_bytes(self._h, int(nsteps), int(ckpt_every), C.byref(nb)))
        return nb.value

    def adjoint(self, nsteps: int, ckpt_every: int = 16, objective: str = "drag", workspace=None):
        """Solver.adjoint for every instance at once (cc_batch_adjoint):
        J (n,) and dJ/d(T_w, Kn, Ma) (n, 3), each instance from its inflow
        Maxwellian.  workspace: a device uint8 tensor of at least
        adjoint_workspace_bytes() bytes to use, else one is allocated."""
        nb = self.adjoint_workspace_bytes(nsteps, ckpt_every)
        if workspace is None:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.solvers[0].device)
        elif workspace.numel() < nb:
            raise ValueError(f"batched adjoint workspace of {workspace.numel()} bytes, {nb} needed")
        n = len(self.solvers)
        out = (C.c_double * (4 * n))()
        self._check(lib().cc_batch_adjoint(self._h, int(nsteps), int(ckpt_every),
                                           0 if objective == "drag" else 1, _ptr(workspace), out))
        a = np.array(out[:]).reshape(n, 4)
        return a[:, 0].copy(), a[:, 1:].copy()

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().cc_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
