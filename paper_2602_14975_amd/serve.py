"""Serving driver: Poisson arrivals of independent replicas into the
continuous-batching server of libnnp (replica_submit / nnp_server_progress /
replica_poll), and the latency and throughput report."""

import ctypes as C
import time

import numpy as np

from . import _abi, nnp


class Server:
    def __init__(self, cons, nc, params, budget_bytes, max_slots):
        self.h = C.c_void_p()
        self.keep = (cons, nc, params)
        _abi.check(nnp.lib().nnp_server_create(cons.handle, nc.handle, C.byref(params), int(budget_bytes),
                                               int(max_slots), C.byref(self.h)))

    def replica_bytes(self, n, box):
        b = C.c_size_t()
        _abi.check(nnp.lib().nnp_server_replica_bytes(self.h, int(n), float(box), C.byref(b)))
        return b.value

    def clock(self):
        return nnp.lib().nnp_server_clock(self.h)

    def replica_submit(self, pos, vel, mass, gamma, species, box, seed, stream_id, n_steps):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        gamma = np.ascontiguousarray(gamma, dtype=np.float64)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        d = _abi.ReplicaDesc(pos.shape[0], pos.ctypes.data_as(C.POINTER(C.c_double)),
                             vel.ctypes.data_as(C.POINTER(C.c_double)), mass.ctypes.data_as(C.POINTER(C.c_double)),
                             gamma.ctypes.data_as(C.POINTER(C.c_double)), sp.ctypes.data_as(C.POINTER(C.c_int32)),
                             float(box), int(seed), int(stream_id), int(n_steps))
        t = C.c_uint64()
        _abi.check(nnp.lib().replica_submit(self.h, C.byref(d), C.byref(t)))
        return t.value

    def replica_poll(self, ticket, n=None):
        st = _abi.ReplicaStatus()
        if n is None:
            _abi.check(nnp.lib().replica_poll(self.h, ticket, C.byref(st), None, None))
            return st, None, None
        pos = np.zeros((n, 3))
        vel = np.zeros((n, 3))
        _abi.check(nnp.lib().replica_poll(self.h, ticket, C.byref(st), pos.ctypes.data_as(C.POINTER(C.c_double)),
                                          vel.ctypes.data_as(C.POINTER(C.c_double))))
        return st, pos, vel

    def progress(self, max_steps=1):
        nres = C.c_int32()
        _abi.check(nnp.lib().nnp_server_progress(self.h, int(max_steps), C.byref(nres)))
        return nres.value

    def latencies(self):
        n = C.c_int64()
        nnp.lib().nnp_server_step_latencies(self.h, None, 0, C.byref(n))
        out = np.zeros(max(n.value, 1))
        nnp.lib().nnp_server_step_latencies(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                            C.byref(n))
        return out[: n.value]

    def close(self):
        if self.h is not None and self.h.value:
            nnp.lib().nnp_server_destroy(self.h)
            self.h = None


def _submit_replica(server, r, k, n_steps, vel_seed_base, gamma_fn, mass_fn):
    import synth
    m = mass_fn(r) if mass_fn else r.standard_masses()
    g = gamma_fn(r) if gamma_fn else np.ones(r.n)
    v = synth.maxwell_boltzmann(m, 300.0, vel_seed_base + k)
    return server.replica_submit(r.pos, v, m, g, r.species, r.box, 4000 + k, k, n_steps)


def saturated_rate(server, replicas, n_steps, steps_per_call=4, vel_seed_base=5000):
    """Closed-loop throughput: every replica submitted at once and the server
    driven while some still wait for admission, i.e. while the budget (or
    the slots) hold the resident set at its limit.  Returns (atom-steps per
    second over that interval, its length in seconds); replicas still
    resident at its end are left to the caller (destroy the server)."""
    t0 = server.clock()
    tickets = [_submit_replica(server, r, k, n_steps, vel_seed_base, None, None) for k, r in enumerate(replicas)]
    while True:
        nres = server.progress(steps_per_call)
        states = [server.replica_poll(t)[0] for t in tickets]
        if nres == 0 or all(st.state != 0 for st in states):
            break
    wall = server.clock() - t0
    atom_steps = sum(st.steps_done * r.n for st, r in zip(states, replicas))
    return atom_steps / wall, wall


def run(server, replicas, arrivals, n_steps, dt_fs, steps_per_call=2, vel_seed_base=5000, gamma_fn=None,
        mass_fn=None, log=None, log_every_s=15.0):
    """Submits replica k at server time arrivals[k] (seconds after start)
    while driving the server `steps_per_call` outer steps per call (each call
    ends at a boundary, where waiting replicas are admitted).  `log`, when
    given, receives a status line every log_every_s seconds.  Returns a
    report."""
    order = np.argsort(arrivals)
    t0 = server.clock()
    tickets = {}
    nxt = 0
    n_total = len(replicas)
    resident_time, last_t, max_res = 0.0, 0.0, 0
    next_log = log_every_s
    while True:
        now = server.clock() - t0
        while nxt < n_total and arrivals[order[nxt]] <= now:
            k = int(order[nxt])
            tickets[k] = _submit_replica(server, replicas[k], k, n_steps, vel_seed_base, gamma_fn, mass_fn)
            nxt += 1
        nres = server.progress(steps_per_call)
        t = server.clock() - t0
        resident_time += nres * (t - last_t)
        last_t = t
        max_res = max(max_res, nres)
        if log and t >= next_log:
            log(f"serving: t = {t:.0f} s, {nxt} of {n_total} submitted, {nres} resident")
            next_log += log_every_s
        if nres == 0:
            if nxt >= n_total:
                # every replica submitted; finished when all are done
                done = all(server.replica_poll(tk)[0].state in (2, 3) for tk in tickets.values())
                if done:
                    break
            else:
                wait = arrivals[order[nxt]] - (server.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
    wall = server.clock() - t0
    lat = server.latencies()
    states = [server.replica_poll(tickets[k])[0] for k in range(n_total)]
    steps = sum(st.steps_done for st in states)
    queue = np.array([st.t_admit - st.t_submit for st in states])
    return {
        "replicas": n_total, "failed": int(sum(st.state == 3 for st in states)), "wall_s": wall,
        "replica_steps": int(steps), "aggregate_ns_per_day": steps * dt_fs * 1e-6 / wall * 86400.0,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3), "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "latency_samples": int(lat.size), "queue_delay_mean_s": float(queue.mean()),
        "queue_delay_p99_s": float(np.percentile(queue, 99)),
        "replicas_waiting_over_1s": int((queue > 1.0).sum()),
        "resident_mean": resident_time / max(wall, 1e-9), "resident_max": int(max_res),
    }
