// Continuous batching of independent replicas (the serving entry points of
// nnp.h).
//
// The server reserves its whole HBM budget once, at creation, as one device
// arena.  Replicas wait in a FIFO host queue; at every outer-step boundary
// the server retires replicas that reached their step count (or failed),
// admits queued ones while a slot is free and the packed layout of the
// resident set still fits the arena, and, when the resident set changed,
// repacks: resident positions and velocities come back to the host, the new
// set is laid out contiguously (block-diagonal neighbour lists, per-replica
// box, Philox key and O-step counter) and uploaded, and forces are
// re-evaluated at the current positions.  Because every kernel is
// atom-centric with a fixed order per atom and per replica, a replica's
// trajectory is bitwise the same alone or in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "common.h"
#include "kernels.h"
#include "model.h"

namespace nnp {

struct Replica {
    uint64_t ticket = 0;
    int64_t n = 0;
    std::vector<double> pos, vel;  // [3][n] on the host while not resident
    std::vector<double> mass, gamma;
    std::vector<int32_t> species;
    double box = 0;
    uint64_t seed = 0, stream_id = 0;
    int n_outer = 0;
    int state = NNP_REPLICA_QUEUED;
    int steps_done = 0;
    nnp_status error = NNP_OK;
    double t_submit = 0, t_admit = 0, t_done = 0, t_last = 0;
    uint64_t step = 0;  // O-steps done
    int64_t cap_cons = 0, cap_nc = 0;
};

struct Server {
    const Model* cons = nullptr;
    const Model* nc = nullptr;
    respa_params p{};
    size_t budget = 0;
    int max_slots = 0;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    std::mutex mu;
    std::deque<Replica*> queue;
    std::vector<Replica*> resident;
    std::unordered_map<uint64_t, std::unique_ptr<Replica>> all;
    uint64_t next_ticket = 1;
    std::vector<double> latencies;
    std::chrono::steady_clock::time_point t0;
    double cap_scale = 1.0;
    // packed layout
    bool packed = false;
    respa_state st{};
    std::vector<int64_t> rep_start;
    std::vector<double> box;
    void* ws = nullptr;
    size_t ws_bytes = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static int64_t list_capacity(int64_t n, double box, double radius, double scale) {
    const double rho = double(n) / (box * box * box);
    const double deg = 4.0 / 3.0 * M_PI * radius * radius * radius * rho;
    return int64_t(std::ceil(double(n) * std::min(deg, double(n)) * 1.5 * scale)) + 256;
}

struct PackedLayout {
    double *pos, *vel, *mass, *gamma, *energy, *pos_ref, *box_dev, *ke;
    int32_t *species, *rep_of_atom;
    float *f_cons, *f_nc;
    int *off_c, *nbr_c, *off_n, *nbr_n;
    char* ws;
    size_t ws_bytes;
};

// Carves the packed arrays of a resident set (null base: measure only).
static size_t carve_packed(Server& sv, const std::vector<Replica*>& set, char* base, size_t cap, PackedLayout& L) {
    int64_t N = 0, Ec = 0, En = 0;
    for (const Replica* r : set) {
        N += r->n;
        Ec += r->cap_cons;
        En += r->cap_nc;
    }
    const int R = int(set.size());
    Arena a(base, cap);
    L.pos = a.take<double>(3 * N);
    L.vel = a.take<double>(3 * N);
    L.mass = a.take<double>(N);
    L.gamma = a.take<double>(N);
    L.species = a.take<int32_t>(N);
    L.rep_of_atom = a.take<int32_t>(N);
    L.f_cons = a.take<float>(3 * N);
    L.f_nc = a.take<float>(3 * N);
    L.energy = a.take<double>(R);
    L.pos_ref = a.take<double>(3 * N);
    L.box_dev = a.take<double>(R);
    L.ke = a.take<double>(R);
    L.off_c = a.take<int>(N + 1);
    L.nbr_c = a.take<int>(Ec);
    L.off_n = a.take<int>(N + 1);
    L.nbr_n = a.take<int>(En);
    const size_t wsb = call_scratch_bytes(sv.cons, sv.nc, std::max<int64_t>(N, 1), std::max(R, 1),
                                          std::max<int64_t>(std::max(Ec, En), 1));
    L.ws = a.take<char>(wsb);
    L.ws_bytes = wsb;
    return a.used;
}

static void set_caps(Server& sv, Replica* r) {
    r->cap_cons = list_capacity(r->n, r->box, sv.cons->desc.cutoff + sv.p.skin, sv.cap_scale);
    r->cap_nc = list_capacity(r->n, r->box, sv.nc->desc.cutoff + sv.p.skin, sv.cap_scale);
}

// Brings the state of the resident replicas back to their host records.
static void download(Server& sv) {
    if (!sv.packed) return;
    const int64_t N = sv.st.sys.n_atoms;
    std::vector<double> pos(3 * N), vel(3 * N);
    NNP_HIP(hipMemcpyAsync(pos.data(), sv.st.pos, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, sv.stream));
    NNP_HIP(hipMemcpyAsync(vel.data(), sv.st.vel, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, sv.stream));
    NNP_HIP(hipStreamSynchronize(sv.stream));
    for (size_t k = 0; k < sv.resident.size(); ++k) {
        Replica* r = sv.resident[k];
        const int64_t a0 = sv.rep_start[k];
        for (int c = 0; c < 3; ++c) {
            std::memcpy(&r->pos[c * r->n], &pos[c * N + a0], sizeof(double) * r->n);
            std::memcpy(&r->vel[c * r->n], &vel[c * N + a0], sizeof(double) * r->n);
        }
    }
}

static void upload(Server& sv) {
    sv.packed = false;
    if (sv.resident.empty()) return;
    PackedLayout L;
    const size_t used = carve_packed(sv, sv.resident, sv.arena, sv.budget, L);
    (void)used;
    const int R = int(sv.resident.size());
    int64_t N = 0, Ec = 0, En = 0;
    sv.rep_start.assign(R + 1, 0);
    sv.box.assign(R, 0.0);
    for (int k = 0; k < R; ++k) {
        const Replica* r = sv.resident[k];
        sv.rep_start[k] = N;
        sv.box[k] = r->box;
        N += r->n;
        Ec += r->cap_cons;
        En += r->cap_nc;
    }
    sv.rep_start[R] = N;
    std::vector<double> pos(3 * N), vel(3 * N), mass(N), gamma(N);
    std::vector<int32_t> species(N), rep(N);
    for (int k = 0; k < R; ++k) {
        const Replica* r = sv.resident[k];
        const int64_t a0 = sv.rep_start[k];
        for (int c = 0; c < 3; ++c) {
            std::memcpy(&pos[c * N + a0], &r->pos[c * r->n], sizeof(double) * r->n);
            std::memcpy(&vel[c * N + a0], &r->vel[c * r->n], sizeof(double) * r->n);
        }
        std::memcpy(&mass[a0], r->mass.data(), sizeof(double) * r->n);
        std::memcpy(&gamma[a0], r->gamma.data(), sizeof(double) * r->n);
        std::memcpy(&species[a0], r->species.data(), sizeof(int32_t) * r->n);
        std::fill(rep.begin() + a0, rep.begin() + a0 + r->n, k);
    }
    hipStream_t s = sv.stream;
    NNP_HIP(hipMemcpyAsync(L.pos, pos.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.vel, vel.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.mass, mass.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.gamma, gamma.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.species, species.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.rep_of_atom, rep.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(L.box_dev, sv.box.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    NNP_HIP(hipStreamSynchronize(s));  // host staging vectors go out of scope
    respa_state& st = sv.st;
    st = respa_state{};
    st.sys.n_atoms = N;
    st.sys.n_rep = R;
    st.sys.pos = L.pos;
    st.sys.species = L.species;
    st.sys.rep_of_atom = L.rep_of_atom;
    st.sys.box_dev = L.box_dev;
    st.sys.rep_start = sv.rep_start.data();
    st.sys.box = sv.box.data();
    st.pos = L.pos;
    st.vel = L.vel;
    st.mass = L.mass;
    st.gamma = L.gamma;
    st.f_cons = L.f_cons;
    st.f_nc = L.f_nc;
    st.energy = L.energy;
    st.pos_ref = L.pos_ref;
    st.nl_cons = nnp_nlist{N, Ec, 0, L.off_c, L.nbr_c, nullptr, sv.cons->desc.cutoff + sv.p.skin};
    st.nl_nc = nnp_nlist{N, En, 0, L.off_n, L.nbr_n, nullptr, sv.nc->desc.cutoff + sv.p.skin};
    st.first_step = 1;
    st.lists_valid = 0;
    st.ke = L.ke;
    sv.ws = L.ws;
    sv.ws_bytes = L.ws_bytes;
    sv.packed = true;
}

static size_t footprint(Server& sv, const std::vector<Replica*>& set) {
    PackedLayout L;
    return carve_packed(sv, set, nullptr, 0, L);
}

// Retire finished or failed replicas and admit queued ones; repack if the
// resident set changed.  Caller holds the mutex.
static void boundary(Server& sv) {
    bool changed = false;
    std::vector<Replica*> keep;
    bool any_leaving = false;
    for (Replica* r : sv.resident)
        any_leaving |= r->state == NNP_REPLICA_FAILED || r->steps_done >= r->n_outer;
    std::vector<Replica*> cand = sv.resident;
    for (Replica* r : sv.resident) {
        if (r->state == NNP_REPLICA_FAILED || r->steps_done >= r->n_outer) continue;
        keep.push_back(r);
    }
    // admission: FIFO while a slot is free and the packed set fits the arena
    std::vector<Replica*> admitted;
    while (!sv.queue.empty() && int(keep.size() + admitted.size()) < sv.max_slots) {
        Replica* r = sv.queue.front();
        std::vector<Replica*> trial = keep;
        trial.insert(trial.end(), admitted.begin(), admitted.end());
        trial.push_back(r);
        if (footprint(sv, trial) > sv.budget) break;
        sv.queue.pop_front();
        admitted.push_back(r);
    }
    if (!any_leaving && admitted.empty()) return;
    changed = true;
    download(sv);  // final or current state of everything resident
    const double t = sv.now();
    for (Replica* r : sv.resident) {
        if (r->state == NNP_REPLICA_FAILED) {
            r->t_done = t;
        } else if (r->steps_done >= r->n_outer) {
            r->state = NNP_REPLICA_DONE;
            r->t_done = r->t_last;
        }
    }
    for (Replica* r : admitted) {
        r->state = NNP_REPLICA_RUNNING;
        r->t_admit = t;
        r->t_last = t;
        keep.push_back(r);
    }
    sv.resident = keep;
    if (changed) upload(sv);
}

}  // namespace nnp

using namespace nnp;

extern "C" nnp_status nnp_server_create(const nnp_model* cons, const nnp_model* nc, const respa_params* params,
                                        size_t hbm_budget_bytes, int32_t max_slots, nnp_server** out) {
    try {
        NNP_REQUIRE(cons && nc && params && out, NNP_EINVAL, "null argument");
        NNP_REQUIRE(max_slots >= 1, NNP_EINVAL, "max_slots must be >= 1");
        NNP_REQUIRE(params->mode == NNP_MODE_DMTS_NC && params->n_inner >= 1, NNP_EINVAL,
                    "the server runs DMTS-NC with n_inner >= 1");
        NNP_REQUIRE(hbm_budget_bytes >= (size_t(1) << 20), NNP_EINVAL, "budget below 1 MiB");
        auto sv = std::make_unique<Server>();
        sv->cons = reinterpret_cast<const Model*>(cons);
        sv->nc = reinterpret_cast<const Model*>(nc);
        NNP_REQUIRE(sv->cons->desc.kind == NNP_MODEL_CONS && sv->nc->desc.kind == NNP_MODEL_NC, NNP_EINVAL,
                    "model kinds do not match");
        sv->p = *params;
        sv->p.check_every = 1;
        sv->p.rewind_threshold = 0.0;  // replicas fail alone; a rewind would move every resident replica
        sv->budget = hbm_budget_bytes;
        sv->max_slots = max_slots;
        sv->t0 = std::chrono::steady_clock::now();
        NNP_HIP(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&sv->arena), hbm_budget_bytes);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(sv->stream);
            set_error(std::string("could not reserve the HBM budget: ") + hipGetErrorString(e));
            return NNP_ENOMEM;
        }
        *out = reinterpret_cast<nnp_server*>(sv.release());
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}

extern "C" void nnp_server_destroy(nnp_server* server) {
    if (!server) return;
    Server* sv = reinterpret_cast<Server*>(server);
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    if (sv->arena) (void)hipFree(sv->arena);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
}

extern "C" nnp_status nnp_server_replica_bytes(const nnp_server* server, int64_t n, double box, size_t* bytes) {
    try {
        NNP_REQUIRE(server && bytes && n >= 1 && box > 0, NNP_EINVAL, "bad argument");
        Server& sv = *const_cast<Server*>(reinterpret_cast<const Server*>(server));
        Replica r;
        r.n = n;
        r.box = box;
        std::lock_guard<std::mutex> lk(sv.mu);
        set_caps(sv, &r);
        *bytes = footprint(sv, {&r});
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}

extern "C" double nnp_server_clock(const nnp_server* server) {
    return server ? reinterpret_cast<const Server*>(server)->now() : 0.0;
}

extern "C" nnp_status replica_submit(nnp_server* server, const replica_desc* d, uint64_t* ticket) {
    try {
        NNP_REQUIRE(server && d && ticket, NNP_EINVAL, "null argument");
        Server& sv = *reinterpret_cast<Server*>(server);
        NNP_REQUIRE(d->n >= 2 && d->pos && d->vel && d->mass && d->gamma && d->species, NNP_EINVAL,
                    "incomplete replica");
        NNP_REQUIRE(d->n_outer_steps >= 1, NNP_EINVAL, "n_outer_steps must be >= 1");
        const double rmax = sv.cons->desc.cutoff + sv.p.skin;
        NNP_REQUIRE(d->box > 2.0 * rmax, NNP_EINVAL, "box edge must exceed twice the Verlet radius");
        auto r = std::make_unique<Replica>();
        r->n = d->n;
        r->pos.resize(3 * d->n);
        r->vel.resize(3 * d->n);
        for (int64_t a = 0; a < d->n; ++a)
            for (int c = 0; c < 3; ++c) {
                r->pos[c * d->n + a] = d->pos[3 * a + c];
                r->vel[c * d->n + a] = d->vel[3 * a + c];
            }
        r->mass.assign(d->mass, d->mass + d->n);
        r->gamma.assign(d->gamma, d->gamma + d->n);
        r->species.assign(d->species, d->species + d->n);
        for (int64_t a = 0; a < d->n; ++a) {
            NNP_REQUIRE(r->species[a] >= 0 && r->species[a] < sv.cons->desc.n_species, NNP_EINVAL,
                        "species out of range");
            NNP_REQUIRE(r->mass[a] > 0, NNP_EINVAL, "masses must be positive");
        }
        r->box = d->box;
        r->seed = d->seed;
        r->stream_id = d->stream_id;
        r->n_outer = d->n_outer_steps;
        std::lock_guard<std::mutex> lk(sv.mu);
        set_caps(sv, r.get());
        NNP_REQUIRE(footprint(sv, {r.get()}) <= sv.budget, NNP_ENOMEM, "replica alone exceeds the HBM budget");
        r->ticket = sv.next_ticket++;
        r->t_submit = sv.now();
        *ticket = r->ticket;
        sv.queue.push_back(r.get());
        sv.all[r->ticket] = std::move(r);
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}

extern "C" nnp_status replica_poll(nnp_server* server, uint64_t ticket, replica_status* out, double* pos_out,
                                   double* vel_out) {
    try {
        NNP_REQUIRE(server && out, NNP_EINVAL, "null argument");
        Server& sv = *reinterpret_cast<Server*>(server);
        std::lock_guard<std::mutex> lk(sv.mu);
        auto it = sv.all.find(ticket);
        NNP_REQUIRE(it != sv.all.end(), NNP_ENOTFOUND, "unknown ticket");
        const Replica& r = *it->second;
        *out = replica_status{r.state, r.steps_done, r.error, r.t_submit, r.t_admit, r.t_done};
        if (r.state == NNP_REPLICA_DONE) {
            for (int64_t a = 0; a < r.n; ++a)
                for (int c = 0; c < 3; ++c) {
                    if (pos_out) pos_out[3 * a + c] = r.pos[c * r.n + a];
                    if (vel_out) vel_out[3 * a + c] = r.vel[c * r.n + a];
                }
        }
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}

extern "C" nnp_status nnp_server_progress(nnp_server* server, int32_t max_outer_steps, int32_t* n_resident) {
    try {
        NNP_REQUIRE(server && max_outer_steps >= 0, NNP_EINVAL, "bad argument");
        Server& sv = *reinterpret_cast<Server*>(server);
        std::lock_guard<std::mutex> lk(sv.mu);
        for (int it = 0; it < max_outer_steps; ++it) {
            boundary(sv);
            if (sv.resident.empty()) break;
            const int R = int(sv.resident.size());
            std::vector<uint64_t> seeds(R), streams(R), base(R);
            std::vector<int> bad(R, 0);
            for (int k = 0; k < R; ++k) {
                seeds[k] = sv.resident[k]->seed;
                streams[k] = sv.resident[k]->stream_id;
                base[k] = sv.resident[k]->step;
            }
            nnp_status e = respa_run(sv.cons, sv.nc, &sv.st, &sv.p, 1, sv.ws, sv.ws_bytes, sv.stream, seeds.data(),
                                     streams.data(), base.data(), bad.data());
            if (e == NNP_ECAPACITY) {
                // state is back at the start of the step: grow every list and repack
                download(sv);
                sv.cap_scale *= 1.5;
                for (Replica* r : sv.resident) set_caps(sv, r);
                std::vector<Replica*> keep;
                for (Replica* r : sv.resident) {
                    if (footprint(sv, {r}) > sv.budget) {
                        r->state = NNP_REPLICA_FAILED;
                        r->error = NNP_ENOMEM;
                        r->t_done = sv.now();
                    } else {
                        keep.push_back(r);
                    }
                }
                while (!keep.empty() && footprint(sv, keep) > sv.budget) {  // requeue the newest
                    Replica* r = keep.back();
                    keep.pop_back();
                    r->state = NNP_REPLICA_QUEUED;
                    sv.queue.push_front(r);
                }
                sv.resident = keep;
                upload(sv);
                continue;
            }
            if (e != NNP_OK) return e;
            const double t = sv.now();
            for (int k = 0; k < R; ++k) {
                Replica* r = sv.resident[k];
                if (bad[k]) {
                    r->state = NNP_REPLICA_FAILED;
                    r->error = NNP_EUNSTABLE;
                    continue;
                }
                sv.latencies.push_back(t - r->t_last);
                r->t_last = t;
                r->steps_done += 1;
                r->step += uint64_t(sv.p.n_inner);
            }
        }
        boundary(sv);
        if (n_resident) *n_resident = int32_t(sv.resident.size());
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}

extern "C" nnp_status nnp_server_step_latencies(nnp_server* server, double* out, int64_t cap, int64_t* n_out) {
    try {
        NNP_REQUIRE(server && n_out, NNP_EINVAL, "null argument");
        Server& sv = *reinterpret_cast<Server*>(server);
        std::lock_guard<std::mutex> lk(sv.mu);
        const int64_t n = int64_t(sv.latencies.size());
        *n_out = n;
        if (out)
            for (int64_t k = 0; k < std::min(n, cap); ++k) out[k] = sv.latencies[k];
    } catch (const Fail& f) {
        return f.code;
    }
    return NNP_OK;
}
