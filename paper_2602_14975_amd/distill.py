"""Distillation of the NC force model onto conservative forces (paper,
Methods "Model training": the small model is fitted to forces labelled by
the large one).

frames:  an NVT single-time-step (BAOAB) trajectory of the conservative
         model; every `every` steps the positions and the conservative forces
         of that configuration are kept (labels come from the same GPU path).
train:   mini-batches of frames packed as independent replicas; force-MSE
         loss and its gradient (nnp_force_mse), weight gradient of the NC
         model (nnp_nc_weight_grad, hand-written reverse pass), FP32 Adam
         (nnp_adam_step).  Returns the validation force RMSE history.
"""

import numpy as np
import torch

from . import nnp


def generate_frames(cons, system, masses, gamma, n_frames, equil_steps, every, dt=0.5, temperature=300.0,
                    seed=4003, vel_seed=5003, skin=1.0, n_traj=1):
    """Frames from `n_traj` independent trajectories (velocity and Philox
    seeds offset by the trajectory index), n_frames / n_traj from each after
    its own equilibration.  Several short runs keep every frame close to the
    starting temperature for teachers whose dynamics drifts over long runs
    (such as randomly initialised ones)."""
    import synth
    assert n_frames % n_traj == 0, "n_frames must be a multiple of n_traj"
    per = n_frames // n_traj
    pos = torch.empty(n_frames, 3, system.n, dtype=torch.float64, device="cuda")
    frc = torch.empty(n_frames, 3, system.n, dtype=torch.float32, device="cuda")
    for t in range(n_traj):
        dev = nnp.DeviceSystem(system.pos, system.species, system.box)
        v0 = synth.maxwell_boltzmann(masses, temperature, vel_seed + t)
        prm = nnp.respa_params(dt, 1, temperature, seed=seed + t, mode="sts", skin=skin, check_every=1)
        traj = nnp.Trajectory(cons, None, dev, v0, masses, gamma, prm)
        if equil_steps > 0:
            traj.respa_step(equil_steps)
        for k in range(per):
            traj.respa_step(every)
            pos[t * per + k].copy_(dev.pos)
            frc[t * per + k].copy_(traj.f_cons)
    return pos, frc


class Distiller:
    def __init__(self, nc, theta0, species, box, n_atoms, batch=16, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.nc = nc
        self.batch = batch
        self.lr, self.betas, self.eps = lr, betas, eps
        self.theta = torch.as_tensor(np.asarray(theta0, dtype=np.float32), device="cuda").clone()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        self.n = n_atoms
        sp = np.asarray(species)
        pos0 = np.zeros((n_atoms, 3))
        self.sys = nnp.DeviceSystem([pos0] * batch, [sp] * batch, [box] * batch)
        cap = int(batch * n_atoms * 4.0 / 3.0 * np.pi * 3.5 ** 3 * 0.2) + 4096
        self.nl = nnp.NeighborList(self.sys.n, nc.cutoff, cap, with_rev=False)
        self.ws = nnp.workspace(None, nc, self.sys.n, batch, cap)
        self.grad_f = torch.empty(3, self.sys.n, dtype=torch.float32, device="cuda")
        self.small_ws = torch.empty(8192, dtype=torch.uint8, device="cuda")

    def _pack(self, pos, frc, idx):
        k = len(idx)
        p = pos[idx].permute(1, 0, 2).reshape(3, k * self.n).contiguous()
        f = frc[idx].permute(1, 0, 2).reshape(3, k * self.n).contiguous()
        return p, f

    def _forces(self, p):
        self.sys.pos.copy_(p)
        nnp.nnp_neighbors(self.sys, self.nl, self.ws)
        return nnp.nnp_nc_forces(self.nc, self.sys, self.nl, self.ws)

    def step(self, pos, frc, idx):
        self.nc.set_weights_f32(self.theta)
        p, f_ref = self._pack(pos, frc, idx)
        f = self._forces(p)
        loss, _ = nnp.nnp_force_mse(f, f_ref, self.small_ws, grad=self.grad_f)
        g = nnp.nnp_nc_weight_grad(self.nc, self.sys, self.nl, self.grad_f, self.ws)
        self.t += 1
        nnp.nnp_adam_step(self.theta, g, self.m, self.v, self.t, self.lr, self.betas[0], self.betas[1], self.eps)
        return loss

    def rmse(self, pos, frc, idx):
        self.nc.set_weights_f32(self.theta)
        tot, cnt = 0.0, 0
        for s0 in range(0, len(idx), self.batch):
            chunk = idx[s0:s0 + self.batch]
            if len(chunk) < self.batch:
                chunk = np.concatenate([chunk, idx[: self.batch - len(chunk)]])
            p, f_ref = self._pack(pos, frc, chunk)
            f = self._forces(p)
            loss, _ = nnp.nnp_force_mse(f, f_ref, self.small_ws)
            tot += float(loss.item()) * f.numel()
            cnt += f.numel()
        return float(np.sqrt(tot / cnt))


def train(nc, theta0, pos, frc, species, box, n_atoms, steps, n_val, batch=16, lr=1e-3, log_every=500, seed=0):
    rng = np.random.default_rng(seed)
    n_frames = pos.shape[0]
    perm = rng.permutation(n_frames)
    val, tr = perm[:n_val], perm[n_val:]
    d = Distiller(nc, theta0, species, box, n_atoms, batch=batch, lr=lr)
    hist = [(0, d.rmse(pos, frc, val))]
    for it in range(1, steps + 1):
        idx = rng.choice(tr, size=batch, replace=False)
        d.step(pos, frc, idx)
        if it % log_every == 0 or it == steps:
            hist.append((it, d.rmse(pos, frc, val)))
    return d, hist
