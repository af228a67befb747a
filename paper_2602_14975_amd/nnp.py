"""Python binding of libnnp: the C entry points under the same names, with
torch tensors as device memory and torch's current HIP stream.

The functions only marshal arguments (pointers, sizes, streams); every step
of the computation runs in the library's HIP kernels.  Device arrays follow
the C layout: positions/velocities float64 [3][n], forces float32 [3][n].
"""

import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import check

DEV = "cuda"


def lib():
    return _abi.load()


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ models --

class Model:
    """Owns an nnp_model (weights on the device, float32)."""

    def __init__(self, kind, width, n_layers, n_rbf, cutoff, weights, n_species=4, n_s=8, n_l=2, n_c=8,
                 poly_p=5, precision=_abi.NNP_FP32):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        self._w = w
        d = _abi.ModelDesc(kind, n_species, width, n_layers, n_rbf, poly_p, n_s, n_l, n_c, precision, cutoff,
                           w.ctypes.data_as(C.POINTER(C.c_double)), w.size)
        h = C.c_void_p()
        check(lib().nnp_model_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.kind, self.width, self.cutoff = kind, width, cutoff
        self.n_weights = int(lib().nnp_model_n_weights(h))

    @classmethod
    def from_spec(cls, spec, weights, precision=_abi.NNP_FP32):
        kind = _abi.NNP_MODEL_CONS if spec.kind == "cons" else _abi.NNP_MODEL_NC
        return cls(kind, spec.width, spec.n_layers, spec.n_rbf, spec.cutoff, weights, spec.n_species, spec.n_s,
                   spec.n_l, spec.n_c, spec.poly_p, precision)

    def set_weights_f32(self, w_dev):
        check(lib().nnp_model_set_weights_f32(self.handle, _ptr(w_dev), w_dev.numel(), _stream()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().nnp_model_destroy(h)
            except Exception:
                pass
            self.handle = None


# ----------------------------------------------------------------- systems --

class DeviceSystem:
    """Packed replicas on the device: pos [3][n] float64, species int32."""

    def __init__(self, pos_list, species_list, boxes, device=DEV):
        if isinstance(pos_list, np.ndarray):
            pos_list, species_list, boxes = [pos_list], [species_list], [boxes]
        sizes = [p.shape[0] for p in pos_list]
        self.rep_start = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.rep_start[1:])
        self.box = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64))
        self.n = int(self.rep_start[-1])
        self.n_rep = len(sizes)
        pos = np.concatenate(pos_list).astype(np.float64)
        sp = np.concatenate(species_list).astype(np.int32)
        if sp.min() < 0:
            raise ValueError("species must be non-negative")
        self.pos = torch.as_tensor(np.ascontiguousarray(pos.T), device=device)
        self.species = torch.as_tensor(sp, device=device)
        rep = np.repeat(np.arange(self.n_rep, dtype=np.int32), sizes)
        self.rep_of_atom = torch.as_tensor(rep, device=device)
        self.box_dev = torch.as_tensor(self.box, device=device)

    def c(self, pos=None):
        """C view; `pos` (device float64 [3][n]) replaces the stored positions."""
        p = self.pos if pos is None else pos
        if p.dtype != torch.float64 or tuple(p.shape) != (3, self.n) or not p.is_contiguous():
            raise ValueError("positions must be a contiguous float64 [3][n] tensor")
        return _abi.System(self.n, self.n_rep, p.data_ptr(), self.species.data_ptr(),
                           self.rep_of_atom.data_ptr() if self.n_rep > 1 else None,
                           self.box_dev.data_ptr() if self.n_rep > 1 else None,
                           self.rep_start.ctypes.data_as(C.POINTER(C.c_int64)),
                           self.box.ctypes.data_as(C.POINTER(C.c_double)))

    def positions(self):
        return self.pos.T.cpu().numpy()


class NeighborList:
    """Caller-owned CSR buffers of an nnp_nlist."""

    def __init__(self, n, cutoff, capacity, with_rev=True, device=DEV):
        self.n, self.cutoff, self.capacity = n, float(cutoff), int(capacity)
        self.offsets = torch.zeros(n + 1, dtype=torch.int32, device=device)
        self.nbr = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.rev = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device) if with_rev else None
        self.n_edges = 0

    def c(self):
        return _abi.NList(self.n, self.capacity, self.n_edges, self.offsets.data_ptr(), self.nbr.data_ptr(),
                          self.rev.data_ptr() if self.rev is not None else None, self.cutoff)

    def grow(self, capacity):
        dev = self.nbr.device
        self.capacity = int(capacity)
        self.nbr = torch.zeros(self.capacity, dtype=torch.int32, device=dev)
        if self.rev is not None:
            self.rev = torch.zeros(self.capacity, dtype=torch.int32, device=dev)

    def rows(self):
        off = self.offsets.cpu().numpy()
        nb = self.nbr.cpu().numpy()
        return off, nb[: off[-1]]


def workspace(cons, nc, n, n_rep, max_edges, device=DEV):
    nbytes = C.c_size_t()
    check(lib().nnp_workspace_size(cons.handle if cons else None, nc.handle if nc else None, n, n_rep, max_edges,
                                   C.byref(nbytes)))
    return torch.empty(nbytes.value, dtype=torch.uint8, device=device)


# ------------------------------------------------------------- entry points --

def nnp_neighbors(system, nlist, ws):
    """Builds nlist at nlist.cutoff; grows the buffers and retries once when
    the capacity is exceeded.  Returns the edge count."""
    for _ in range(2):
        cl = nlist.c()
        code = lib().nnp_neighbors(C.byref(system.c()), C.byref(cl), _ptr(ws), ws.numel(), _stream())
        nlist.n_edges = int(cl.n_edges)
        if code == _abi.NNP_ECAPACITY and cl.n_edges > nlist.capacity:
            nlist.grow(int(cl.n_edges * 1.2) + 64)
            continue
        check(code)
        return nlist.n_edges
    raise RuntimeError("neighbour list did not fit after growing")


def nnp_cons_energy_forces(model, system, nlist, ws, energy=None, forces=None):
    energy = energy if energy is not None else torch.empty(system.n_rep, dtype=torch.float64, device=DEV)
    forces = forces if forces is not None else torch.empty(3, system.n, dtype=torch.float32, device=DEV)
    check(lib().nnp_cons_energy_forces(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(ws),
                                       ws.numel(), _ptr(energy), _ptr(forces), _stream()))
    return energy, forces


def nnp_nc_forces(model, system, nlist, ws, forces=None):
    forces = forces if forces is not None else torch.empty(3, system.n, dtype=torch.float32, device=DEV)
    check(lib().nnp_nc_forces(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(ws), ws.numel(),
                              _ptr(forces), _stream()))
    return forces


def nnp_nc_forces_noalloc(model, system, nlist, forces=None):
    """nnp_nc_forces without a workspace: the library's static device scratch
    (nnp_nc_forces_noalloc_max_bytes() bytes) serves the call."""
    forces = forces if forces is not None else torch.empty(3, system.n, dtype=torch.float32, device=DEV)
    check(lib().nnp_nc_forces_noalloc(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(forces),
                                      _stream()))
    return forces


def nnp_cons_virial(model, system, nlist, ws):
    """(energy [n_rep], forces [3][n], virial W = -sum F . q [n_rep])."""
    energy = torch.empty(system.n_rep, dtype=torch.float64, device=DEV)
    forces = torch.empty(3, system.n, dtype=torch.float32, device=DEV)
    virial = torch.empty(system.n_rep, dtype=torch.float64, device=DEV)
    check(lib().nnp_cons_virial(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(ws), ws.numel(),
                                _ptr(energy), _ptr(forces), _ptr(virial), _stream()))
    return energy, forces, virial


def nnp_nc_virial(model, system, nlist, ws):
    """(forces [3][n], virial proxy sum F_ij . r_ij [n_rep])."""
    forces = torch.empty(3, system.n, dtype=torch.float32, device=DEV)
    virial = torch.empty(system.n_rep, dtype=torch.float64, device=DEV)
    check(lib().nnp_nc_virial(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(ws), ws.numel(),
                              _ptr(forces), _ptr(virial), _stream()))
    return forces, virial


def nnp_nc_weight_grad(model, system, nlist, dl_df, ws, out=None):
    out = out if out is not None else torch.empty(model.n_weights, dtype=torch.float32, device=DEV)
    dl_df = dl_df.contiguous()
    check(lib().nnp_nc_weight_grad(model.handle, C.byref(system.c()), C.byref(nlist.c()), _ptr(dl_df), _ptr(out),
                                   _ptr(ws), ws.numel(), _stream()))
    return out


def nnp_force_mse(f, f_ref, ws, grad=None):
    """Returns (loss float64 [1], grad) with grad = 2 (f - f_ref) / f.numel()."""
    loss = torch.empty(1, dtype=torch.float64, device=f.device)
    check(lib().nnp_force_mse(_ptr(f), _ptr(f_ref), f.numel(), _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(),
                              _stream()))
    return loss, grad


def nnp_adam_step(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    check(lib().nnp_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), int(t), lr, beta1, beta2,
                              eps, _stream()))


def nnp_hmr_masses(bonded_heavy, masses, h_mass=3.0, mode="set"):
    bh = np.ascontiguousarray(bonded_heavy, dtype=np.int32)
    m = np.ascontiguousarray(masses, dtype=np.float64)
    out = np.empty_like(m)
    check(lib().nnp_hmr_masses(m.size, bh.ctypes.data_as(C.POINTER(C.c_int32)),
                               m.ctypes.data_as(C.POINTER(C.c_double)), float(h_mass), 0 if mode == "set" else 1,
                               out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


# -------------------------------------------------------------- trajectory --

class Trajectory:
    """Device-resident respa_state plus its list buffers and workspace."""

    def __init__(self, cons, nc, system, vel, masses, gamma, params, skin=1.0, capacity_factor=1.4,
                 virial=False, cell_order=True):
        """cell_order: the force evaluations keep their rows in the cell order
        of each list build (respa_state.order); the results are the same bits
        either way."""
        self.cons, self.nc, self.sys = cons, nc, system
        n = system.n
        self.params = params
        self.dmts = params.mode in (_abi.NNP_MODE_DMTS_NC, _abi.NNP_MODE_DMTS)
        self.vel = torch.as_tensor(np.ascontiguousarray(np.asarray(vel, dtype=np.float64).T), device=DEV)
        self.mass = torch.as_tensor(np.asarray(masses, dtype=np.float64), device=DEV)
        self.gamma = torch.as_tensor(np.asarray(gamma, dtype=np.float64), device=DEV)
        self.f_cons = torch.zeros(3, n, dtype=torch.float32, device=DEV)
        self.f_nc = torch.zeros(3, n, dtype=torch.float32, device=DEV)
        self.energy = torch.zeros(system.n_rep, dtype=torch.float64, device=DEV)
        self.pos_ref = torch.zeros(3, n, dtype=torch.float64, device=DEV)
        # NPT virial estimator of the last outer step, per replica (respa_step)
        self.virial = torch.zeros(system.n_rep, dtype=torch.float64, device=DEV) if virial else None
        self.order = torch.zeros(2 * n, dtype=torch.int32, device=DEV) if cell_order else None
        # initial capacity from a list build at the Verlet radius
        ws0 = workspace(None, None, n, system.n_rep, 1)
        rc_c = cons.cutoff + params.skin
        probe = NeighborList(n, rc_c, 1, with_rev=False)
        cl = probe.c()
        lib().nnp_neighbors(C.byref(system.c()), C.byref(cl), _ptr(ws0), ws0.numel(), _stream())
        cap = int(cl.n_edges * capacity_factor) + 1024
        self.nl_cons = NeighborList(n, rc_c, cap, with_rev=False)
        if self.dmts:
            rc_n = nc.cutoff + params.skin
            self.nl_nc = NeighborList(n, rc_n, max(int(cap * (rc_n / rc_c) ** 3 * 1.2), 1024), with_rev=False)
        else:
            self.nl_nc = NeighborList(n, 0.0, 1, with_rev=False)
        self.ws = workspace(cons, nc if self.dmts else None, n, system.n_rep, cap)
        self.step_count = 0
        self.first_step = 1
        self.lists_valid = 0
        self.n_rebuilds = 0
        self.n_rewinds = 0
        self.n_replays = 0

    def _state(self, ke):
        return _abi.RespaState(self.sys.c(), self.sys.pos.data_ptr(), self.vel.data_ptr(), self.mass.data_ptr(),
                               self.gamma.data_ptr(), self.f_cons.data_ptr(), self.f_nc.data_ptr(),
                               self.energy.data_ptr(), self.pos_ref.data_ptr(), self.nl_cons.c(), self.nl_nc.c(),
                               self.step_count, self.first_step, self.lists_valid,
                               ke.data_ptr() if ke is not None else None, self.n_rebuilds, self.n_rewinds,
                               self.n_replays, self.virial.data_ptr() if self.virial is not None else None,
                               self.order.data_ptr() if self.order is not None else None)

    def respa_step(self, n_outer, ke=None):
        """Advances by n_outer outer steps, growing the list buffers on
        NNP_ECAPACITY (each retry resumes at the failed outer step; growth is
        by 1.3x the reported need, so a second retry means the lists kept
        growing).  NNP_EROWLIMIT and every other error raise at once.
        ke: optional float64 [n_outer][n_rep] tensor."""
        for _ in range(8):
            st = self._state(ke)
            code = lib().respa_step(self.cons.handle, self.nc.handle if self.nc else None, C.byref(st),
                                    C.byref(self.params), int(n_outer), _ptr(self.ws), self.ws.numel(), _stream())
            done = int(st.step) - self.step_count
            self.step_count = int(st.step)
            self.first_step = int(st.first_step)
            self.lists_valid = int(st.lists_valid)
            self.n_rebuilds = int(st.n_rebuilds)
            self.n_rewinds = int(st.n_rewinds)
            self.n_replays = int(st.n_replays)
            if code == _abi.NNP_ECAPACITY:
                need_c, need_n = int(st.nl_cons.n_edges), int(st.nl_nc.n_edges)
                if need_c > self.nl_cons.capacity:
                    self.nl_cons.grow(int(need_c * 1.3) + 1024)
                if need_n > self.nl_nc.capacity:
                    self.nl_nc.grow(int(need_n * 1.3) + 1024)
                self.ws = workspace(self.cons, self.nc if self.dmts else None, self.sys.n, self.sys.n_rep,
                                    max(self.nl_cons.capacity, self.nl_nc.capacity))
                n_in = max(1, self.params.n_inner) if self.dmts else 1
                n_outer -= done // n_in
                if n_outer <= 0:
                    return
                continue
            check(code)
            return
        raise RuntimeError("respa_step: list capacity was exceeded 8 times in a row although each retry grew "
                           "the buffers to 1.3x the reported need; the system is probably collapsing")

    def barostat(self, params, step):
        """One stochastic cell rescaling step (nnp_barostat_scr) fed by the
        virial estimator of the last outer step; updates the system's box
        edges in place.  Needs virial=True."""
        if self.virial is None:
            raise ValueError("the barostat needs a trajectory created with virial=True")
        st = self._state(None)
        box_dev = self.sys.box_dev.data_ptr()
        check(lib().nnp_barostat_scr(C.byref(st), C.byref(params), int(step),
                                     self.sys.box.ctypes.data_as(C.c_void_p), box_dev, _ptr(self.ws),
                                     self.ws.numel(), _stream()))
        self.first_step = int(st.first_step)
        self.lists_valid = int(st.lists_valid)
        return self.sys.box.copy()

    def positions(self):
        return self.sys.pos.T.cpu().numpy()

    def velocities(self):
        return self.vel.T.cpu().numpy()


_MODES = {"dmts_nc": _abi.NNP_MODE_DMTS_NC, "sts": _abi.NNP_MODE_STS, "dmts": _abi.NNP_MODE_DMTS}


def barostat_params(pressure_bar=1.0, compressibility_per_bar=4.5e-5, tau_fs=100.0, dt_fs=4.0, temperature=300.0,
                    seed=6000, stream_id=0):
    return _abi.BarostatParams(float(pressure_bar), float(compressibility_per_bar), float(tau_fs), float(dt_fs),
                               float(temperature), int(seed), int(stream_id))


def respa_params(dt_outer, n_inner, temperature=300.0, seed=4000, stream_id=0, mode="dmts_nc", thermostat="langevin",
                 skin=1.0, check_every=1, rewind_threshold=0.0, save_every=1, sts_after_rewind=0, graph=True):
    return _abi.RespaParams(float(dt_outer), int(n_inner), _MODES[mode],
                            _abi.NNP_THERMO_FFL if thermostat == "ffl" else _abi.NNP_THERMO_LANGEVIN,
                            int(check_every), float(temperature), int(seed), int(stream_id), float(skin),
                            float(rewind_threshold), int(save_every), int(sts_after_rewind), int(bool(graph)))
