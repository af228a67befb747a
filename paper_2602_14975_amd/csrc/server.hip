// Continuous batching of independent replicas (the serving entry points of
// nnp.h).
//
// The server reserves its whole HBM budget once, at creation, as one device
// arena.  Its fixed part holds two banks of packed per-atom state (positions,
// velocities, masses, frictions, species, cached forces F and F_NC) sized
// for the most atoms the budget can ever hold, a staging bank for replicas
// being admitted, and the step timestamps; the rest of the arena holds the
// neighbour lists and the evaluation scratch of the current resident set.
//
// Replicas wait in a FIFO host queue.  At an outer-step boundary the server
// retires replicas that reached their step count (or failed), copying only
// their final state to the host, and admits queued ones while a slot is free
// and the resident set still fits the budget.  Admitted replicas are
// uploaded once into the staging bank, where their lists are built and F
// and F_NC evaluated (the first step of Algorithm 1).  A gather kernel then
// writes the new packed layout into the other bank: resident replicas move
// device to device with their cached forces, admitted ones come from the
// staging bank; nothing resident goes through the host and nothing is
// evaluated again.  Lists are rebuilt for the new layout at the next step.
//
// Between boundaries the resident set advances by several outer steps in
// one call of the integrator (recorded outer steps replayed as a graph,
// one status check at the end).  Each outer step ends with a device
// timestamp, so the per-replica step latency (time between consecutive step
// completions, the first from the admission) is measured on the device
// clock.  Every kernel is atom-centric with a fixed order per atom and per
// replica, so a replica's trajectory is bitwise the same alone or in any mix.
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

constexpr int kMaxStepsPerCall = 64;

struct Replica {
    uint64_t ticket = 0;
    int64_t n = 0;
    std::vector<double> pos, vel;  // [3][n] on the host: the submitted, then the final state
    std::vector<double> mass, gamma;
    std::vector<int32_t> species;
    double box = 0;
    uint64_t seed = 0, stream_id = 0;
    int n_outer = 0;
    int state = NNP_REPLICA_QUEUED;
    int steps_done = 0;
    nnp_status error = NNP_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t tick_last = 0;  // device clock of the last step completion (or of the admission)
    uint64_t step = 0;       // O-steps done
    int64_t cap_cons = 0, cap_nc = 0;
};

// Packed per-atom state, [3][N] or [N] with N the atoms of the layout.
struct Bank {
    double *pos = nullptr, *vel = nullptr, *mass = nullptr, *gamma = nullptr, *energy = nullptr,
           *box_dev = nullptr;
    int32_t *species = nullptr, *rep_of_atom = nullptr;
    float *f_cons = nullptr, *f_nc = nullptr;
};

// One entry per destination replica of a repack.
struct RepackEntry {
    int64_t dst_start, src_start, n;
    int32_t src_bank;  // 0: the current bank, 1: the staging bank
    int32_t src_rep;   // replica index within the source layout
    double box;
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
    double tick_hz = 1e8;
    // fixed part of the arena
    int64_t n_cap = 0;
    size_t fixed_bytes = 0;
    Bank bank[2], staging;
    int cur = 0;
    double* pos_ref = nullptr;
    uint64_t* stamps = nullptr;  // [kMaxStepsPerCall + 1]: the steps of a call, then an admission
    RepackEntry* repack_dev = nullptr;
    // current packed layout
    bool packed = false;
    respa_state st{};
    std::vector<int64_t> rep_start;
    std::vector<double> box;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // pinned host mirrors for the step timestamps and the repack table
    uint64_t* stamps_host = nullptr;
    RepackEntry* repack_host = nullptr;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static int64_t list_capacity(int64_t n, double box, double radius, double scale) {
    const double rho = double(n) / (box * box * box);
    const double deg = 4.0 / 3.0 * M_PI * radius * radius * radius * rho;
    return int64_t(std::ceil(double(n) * std::min(deg, double(n)) * 1.5 * scale)) + 256;
}

static void carve_bank(Arena& a, int64_t N, int R, Bank& b) {
    b.pos = a.take<double>(3 * N);
    b.vel = a.take<double>(3 * N);
    b.mass = a.take<double>(N);
    b.gamma = a.take<double>(N);
    b.species = a.take<int32_t>(N);
    b.rep_of_atom = a.take<int32_t>(N);
    b.f_cons = a.take<float>(3 * N);
    b.f_nc = a.take<float>(3 * N);
    b.energy = a.take<double>(R);
    b.box_dev = a.take<double>(R);
}

static void carve_fixed(Server& sv, int64_t n_cap, Arena& a) {
    carve_bank(a, n_cap, sv.max_slots, sv.bank[0]);
    carve_bank(a, n_cap, sv.max_slots, sv.bank[1]);
    carve_bank(a, n_cap, sv.max_slots, sv.staging);
    sv.pos_ref = a.take<double>(3 * n_cap);
    sv.stamps = a.take<uint64_t>(kMaxStepsPerCall + 1);
    sv.repack_dev = a.take<RepackEntry>(sv.max_slots);
}

struct Dynamic {
    int *off_c, *nbr_c, *off_n, *nbr_n;
    int* order;  // [2N]: the cell order of the evaluations' rows (respa_state.order)
    char* ws;
    size_t ws_bytes;
};

// Lists and evaluation scratch of a set, after the fixed part (null base:
// measure only).  Returns the bytes of the whole arena in use.
static size_t carve_dynamic(Server& sv, const std::vector<Replica*>& set, char* base, Dynamic& D) {
    int64_t N = 0, Ec = 0, En = 0;
    for (const Replica* r : set) {
        N += r->n;
        Ec += r->cap_cons;
        En += r->cap_nc;
    }
    const int R = int(set.size());
    Arena a(base, base ? sv.budget : 0);
    a.used = sv.fixed_bytes;
    D.off_c = a.take<int>(N + 1);
    D.nbr_c = a.take<int>(Ec);
    D.off_n = a.take<int>(N + 1);
    D.nbr_n = a.take<int>(En);
    D.order = a.take<int>(2 * std::max<int64_t>(N, 1));
    const size_t wsb = call_scratch_bytes(sv.cons, sv.nc, std::max<int64_t>(N, 1), std::max(R, 1),
                                          std::max<int64_t>(std::max(Ec, En), 1));
    D.ws = a.take<char>(wsb);
    D.ws_bytes = wsb;
    return a.used;
}

static bool fits(Server& sv, const std::vector<Replica*>& set) {
    int64_t N = 0;
    for (const Replica* r : set) N += r->n;
    if (N > sv.n_cap || int(set.size()) > sv.max_slots) return false;
    Dynamic D;
    return carve_dynamic(sv, set, nullptr, D) <= sv.budget;
}

static void set_caps(Server& sv, Replica* r) {
    r->cap_cons = list_capacity(r->n, r->box, sv.cons->desc.cutoff + sv.p.skin, sv.cap_scale);
    r->cap_nc = list_capacity(r->n, r->box, sv.nc->desc.cutoff + sv.p.skin, sv.cap_scale);
}

// Gathers the new packed layout into `dst`: replica k' of the new layout
// copies its atoms from the current bank or the staging bank.
__global__ void k_repack(const RepackEntry* __restrict__ map, Bank cur, int64_t n_cur, Bank stg, int64_t n_stg,
                         Bank dst, int64_t n_dst) {
    const int k = blockIdx.y;
    const RepackEntry e = map[k];
    const Bank& src = e.src_bank ? stg : cur;
    const int64_t ns = e.src_bank ? n_stg : n_cur;
    for (int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; a < e.n; a += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = e.src_start + a, j = e.dst_start + a;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dst.pos[c * n_dst + j] = src.pos[c * ns + i];
            dst.vel[c * n_dst + j] = src.vel[c * ns + i];
            dst.f_cons[c * n_dst + j] = src.f_cons[c * ns + i];
            dst.f_nc[c * n_dst + j] = src.f_nc[c * ns + i];
        }
        dst.mass[j] = src.mass[i];
        dst.gamma[j] = src.gamma[i];
        dst.species[j] = src.species[i];
        dst.rep_of_atom[j] = k;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dst.energy[k] = src.energy[e.src_rep];
        dst.box_dev[k] = e.box;
    }
}

// Points the state at bank `b` for the layout (rep_start, box) with the
// current dynamic part.
static void point_state(Server& sv, const Bank& b, const Dynamic& D, int64_t Ec, int64_t En) {
    const int R = int(sv.rep_start.size()) - 1;
    const int64_t N = sv.rep_start[R];
    respa_state& st = sv.st;
    st = respa_state{};
    st.sys.n_atoms = N;
    st.sys.n_rep = R;
    st.sys.pos = b.pos;
    st.sys.species = b.species;
    st.sys.rep_of_atom = b.rep_of_atom;
    st.sys.box_dev = b.box_dev;
    st.sys.rep_start = sv.rep_start.data();
    st.sys.box = sv.box.data();
    st.pos = b.pos;
    st.vel = b.vel;
    st.mass = b.mass;
    st.gamma = b.gamma;
    st.f_cons = b.f_cons;
    st.f_nc = b.f_nc;
    st.energy = b.energy;
    st.pos_ref = sv.pos_ref;
    st.nl_cons = nnp_nlist{N, Ec, 0, D.off_c, D.nbr_c, nullptr, sv.cons->desc.cutoff + sv.p.skin};
    st.nl_nc = nnp_nlist{N, En, 0, D.off_n, D.nbr_n, nullptr, sv.nc->desc.cutoff + sv.p.skin};
    st.order = D.order;  // rebuilt with the lists (lists_valid = 0)
    st.lists_valid = 0;
    st.first_step = 0;
    sv.ws = D.ws;
    sv.ws_bytes = D.ws_bytes;
}

static void sums(const std::vector<Replica*>& set, int64_t& N, int64_t& Ec, int64_t& En) {
    N = Ec = En = 0;
    for (const Replica* r : set) {
        N += r->n;
        Ec += r->cap_cons;
        En += r->cap_nc;
    }
}

// Uploads `adm` into the staging bank and evaluates F and F_NC there (lists
// built in the dynamic part, which is carved for a superset).  Returns
// NNP_ECAPACITY when a list outgrew its estimate.
static nnp_status stage(Server& sv, const std::vector<Replica*>& adm, const Dynamic& D) {
    int64_t N, Ec, En;
    sums(adm, N, Ec, En);
    const int R = int(adm.size());
    std::vector<int64_t> rs(R + 1, 0);
    std::vector<double> bx(R);
    std::vector<int32_t> rep(N);
    std::vector<double> pos(3 * N), vel(3 * N), mass(N), gamma(N);
    std::vector<int32_t> species(N);
    for (int k = 0; k < R; ++k) {
        const Replica* r = adm[k];
        rs[k + 1] = rs[k] + r->n;
        bx[k] = r->box;
        const int64_t a0 = rs[k];
        for (int c = 0; c < 3; ++c) {
            std::memcpy(&pos[c * N + a0], &r->pos[c * r->n], sizeof(double) * r->n);
            std::memcpy(&vel[c * N + a0], &r->vel[c * r->n], sizeof(double) * r->n);
        }
        std::memcpy(&mass[a0], r->mass.data(), sizeof(double) * r->n);
        std::memcpy(&gamma[a0], r->gamma.data(), sizeof(double) * r->n);
        std::memcpy(&species[a0], r->species.data(), sizeof(int32_t) * r->n);
        std::fill(rep.begin() + a0, rep.begin() + a0 + r->n, k);
    }
    const Bank& b = sv.staging;
    hipStream_t s = sv.stream;
    NNP_HIP(hipMemcpyAsync(b.pos, pos.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.vel, vel.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.mass, mass.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.gamma, gamma.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.species, species.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.rep_of_atom, rep.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(b.box_dev, bx.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    respa_state st{};
    st.sys.n_atoms = N;
    st.sys.n_rep = R;
    st.sys.pos = b.pos;
    st.sys.species = b.species;
    st.sys.rep_of_atom = b.rep_of_atom;
    st.sys.box_dev = b.box_dev;
    st.sys.rep_start = rs.data();
    st.sys.box = bx.data();
    st.pos = b.pos;
    st.vel = b.vel;
    st.mass = b.mass;
    st.gamma = b.gamma;
    st.f_cons = b.f_cons;
    st.f_nc = b.f_nc;
    st.energy = b.energy;
    st.pos_ref = sv.pos_ref;
    st.nl_cons = nnp_nlist{N, Ec, 0, D.off_c, D.nbr_c, nullptr, sv.cons->desc.cutoff + sv.p.skin};
    st.nl_nc = nnp_nlist{N, En, 0, D.off_n, D.nbr_n, nullptr, sv.nc->desc.cutoff + sv.p.skin};
    st.first_step = 1;
    st.lists_valid = 0;
    std::vector<uint64_t> seeds(R), streams(R), base(R);
    for (int k = 0; k < R; ++k) {
        seeds[k] = adm[k]->seed;
        streams[k] = adm[k]->stream_id;
        base[k] = adm[k]->step;
    }
    std::vector<int> bad(R, 0);
    // zero outer steps: build the lists and evaluate F and F_NC, then check
    nnp_status e = respa_run(sv.cons, sv.nc, &st, &sv.p, 0, D.ws, D.ws_bytes, s, seeds.data(), streams.data(),
                             base.data(), bad.data());
    if (e == NNP_OK) {
        for (int k = 0; k < R; ++k)
            if (bad[k]) {
                adm[k]->state = NNP_REPLICA_FAILED;
                adm[k]->error = NNP_EUNSTABLE;
            }
    }
    return e;
}

// Copies the final state of resident replica k (current layout) to its host record.
static void download_one(Server& sv, int k) {
    Replica* r = sv.resident[k];
    const int64_t N = sv.st.sys.n_atoms, a0 = sv.rep_start[k];
    for (int c = 0; c < 3; ++c) {
        NNP_HIP(hipMemcpyAsync(&r->pos[c * r->n], sv.st.pos + c * N + a0, sizeof(double) * r->n,
                               hipMemcpyDeviceToHost, sv.stream));
        NNP_HIP(hipMemcpyAsync(&r->vel[c * r->n], sv.st.vel + c * N + a0, sizeof(double) * r->n,
                               hipMemcpyDeviceToHost, sv.stream));
    }
}

// Retire finished or failed replicas and admit queued ones; when the
// resident set changed, repack on the device.  Caller holds the mutex.
static void boundary(Server& sv) {
    std::vector<Replica*> keep;
    bool any_leaving = false;
    for (Replica* r : sv.resident) {
        if (r->state == NNP_REPLICA_FAILED || r->steps_done >= r->n_outer) {
            any_leaving = true;
        } else {
            keep.push_back(r);
        }
    }
    // a queue head that no longer fits even alone (list estimates grew) fails
    while (keep.empty() && !sv.queue.empty() && !fits(sv, {sv.queue.front()})) {
        Replica* r = sv.queue.front();
        sv.queue.pop_front();
        r->state = NNP_REPLICA_FAILED;
        r->error = NNP_ENOMEM;
        r->t_done = sv.now();
    }
    std::vector<Replica*> admitted;
    for (;;) {
        // admission: FIFO while a slot is free and the resident set fits
        admitted.clear();
        std::vector<Replica*> trial = keep;
        for (Replica* r : sv.queue) {
            if (int(trial.size()) >= sv.max_slots) break;
            trial.push_back(r);
            if (!fits(sv, trial)) break;
            admitted.push_back(r);
        }
        if (!any_leaving && admitted.empty()) return;
        std::vector<Replica*> next = keep;
        next.insert(next.end(), admitted.begin(), admitted.end());
        Dynamic D;
        carve_dynamic(sv, next, sv.arena, D);
        if (!admitted.empty()) {
            const nnp_status e = stage(sv, admitted, D);
            if (e == NNP_ECAPACITY) {
                // a list outgrew its estimate: larger estimates, admit again
                sv.cap_scale *= 1.5;
                for (Replica* r : sv.resident) set_caps(sv, r);
                for (Replica* r : sv.queue) set_caps(sv, r);
                std::vector<Replica*> still;
                for (Replica* r : keep) {
                    if (fits(sv, {r})) {
                        still.push_back(r);
                    } else {
                        r->state = NNP_REPLICA_FAILED;
                        r->error = NNP_ENOMEM;
                        any_leaving = true;
                    }
                }
                keep = still;
                continue;
            }
            if (e != NNP_OK) throw Fail{e};
        }
        // retiring replicas: final state to the host
        const double t = sv.now();
        std::vector<Replica*> leaving;
        for (size_t k = 0; k < sv.resident.size(); ++k) {
            Replica* r = sv.resident[k];
            if (std::find(keep.begin(), keep.end(), r) != keep.end()) continue;
            download_one(sv, int(k));
            leaving.push_back(r);
        }
        // the new layout: resident replicas first (in order), then admitted ones
        const int R = int(next.size());
        std::vector<int64_t> rs(R + 1, 0);
        std::vector<double> bx(R);
        int64_t n_stg = 0;
        for (Replica* r : admitted) n_stg += r->n;
        int64_t stg_off = 0;
        int stg_rep = 0;
        for (int k = 0; k < R; ++k) {
            Replica* r = next[k];
            rs[k + 1] = rs[k] + r->n;
            bx[k] = r->box;
            RepackEntry& e = sv.repack_host[k];
            e.dst_start = rs[k];
            e.n = r->n;
            e.box = r->box;
            if (k < int(keep.size())) {
                const int old = int(std::find(sv.resident.begin(), sv.resident.end(), r) - sv.resident.begin());
                e.src_bank = 0;
                e.src_start = sv.rep_start[old];
                e.src_rep = old;
            } else {
                e.src_bank = 1;
                e.src_start = stg_off;
                e.src_rep = stg_rep++;
                stg_off += r->n;
            }
        }
        const int dst = sv.cur ^ 1;
        if (R > 0) {
            NNP_HIP(hipMemcpyAsync(sv.repack_dev, sv.repack_host, sizeof(RepackEntry) * R, hipMemcpyHostToDevice,
                                   sv.stream));
            int64_t nmax = 1;
            for (Replica* r : next) nmax = std::max(nmax, r->n);
            const dim3 grid(unsigned(std::min<int64_t>(cdiv(nmax, 256), 64)), unsigned(R));
            const int64_t n_cur = sv.packed ? sv.st.sys.n_atoms : 0;
            k_repack<<<grid, 256, 0, sv.stream>>>(sv.repack_dev, sv.bank[sv.cur], n_cur, sv.staging, n_stg,
                                                  sv.bank[dst], rs[R]);
            NNP_LAUNCH_CHECK();
            if (!admitted.empty()) launch_stamp(sv.stamps + kMaxStepsPerCall, sv.stream);
        }
        NNP_HIP(hipMemcpyAsync(sv.stamps_host + kMaxStepsPerCall, sv.stamps + kMaxStepsPerCall, sizeof(uint64_t),
                               hipMemcpyDeviceToHost, sv.stream));
        NNP_HIP(hipStreamSynchronize(sv.stream));
        for (Replica* r : leaving) {
            if (r->state == NNP_REPLICA_FAILED) {
                r->t_done = t;
            } else {
                r->state = NNP_REPLICA_DONE;
                r->t_done = t;
            }
        }
        for (Replica* r : admitted) {
            sv.queue.erase(std::find(sv.queue.begin(), sv.queue.end(), r));
            if (r->state == NNP_REPLICA_FAILED) continue;  // not finite after its first evaluation
            r->state = NNP_REPLICA_RUNNING;
            r->t_admit = t;
            r->tick_last = sv.stamps_host[kMaxStepsPerCall];
        }
        sv.resident = next;
        sv.cur = dst;
        sv.rep_start = rs;
        sv.box = bx;
        sv.packed = R > 0;
        if (sv.packed) {
            int64_t N, Ec, En;
            sums(next, N, Ec, En);
            point_state(sv, sv.bank[dst], D, Ec, En);
        }
        // a replica found not finite at admission leaves at the next boundary
        return;
    }
}

// Grows every list estimate after a capacity failure of the resident set
// (its state is back at the start of the failed call) and re-carves; the
// newest replicas fail when the set no longer fits and leave through a
// boundary.
static void grow_lists(Server& sv) {
    sv.cap_scale *= 1.5;
    for (Replica* r : sv.resident) set_caps(sv, r);
    for (Replica* r : sv.queue) set_caps(sv, r);
    std::vector<Replica*> keep;
    for (Replica* r : sv.resident) {
        if (fits(sv, {r})) {
            keep.push_back(r);
        } else {
            r->state = NNP_REPLICA_FAILED;
            r->error = NNP_ENOMEM;
        }
    }
    while (keep.size() > 1 && !fits(sv, keep)) {
        keep.back()->state = NNP_REPLICA_FAILED;
        keep.back()->error = NNP_ENOMEM;
        keep.pop_back();
    }
    if (keep.size() != sv.resident.size()) {
        boundary(sv);
        return;
    }
    int64_t N, Ec, En;
    sums(sv.resident, N, Ec, En);
    Dynamic D;
    carve_dynamic(sv, sv.resident, sv.arena, D);
    point_state(sv, sv.bank[sv.cur], D, Ec, En);
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
        sv->p.rewind_threshold = 0.0;  // replicas fail alone; a rewind would move every resident replica
        sv->budget = hbm_budget_bytes;
        sv->max_slots = max_slots;
        sv->t0 = std::chrono::steady_clock::now();
        // the most atoms the budget can hold: per atom the three banks and
        // pos_ref, plus the smallest scratch an atom can need (no edges)
        {
            const int64_t probe = 65536;
            const double per_atom =
                3.0 * (48 + 16 + 8 + 24) + 24 + 8 +
                double(call_scratch_bytes(sv->cons, sv->nc, probe, 1, 1)) / double(probe);
            sv->n_cap = int64_t(double(hbm_budget_bytes) / per_atom);
            NNP_REQUIRE(sv->n_cap >= 2, NNP_EINVAL, "budget too small for any replica");
            Arena a(nullptr, 0);
            carve_fixed(*sv, sv->n_cap, a);
            sv->fixed_bytes = a.used;
            NNP_REQUIRE(sv->fixed_bytes < hbm_budget_bytes, NNP_EINVAL, "budget too small for any replica");
        }
        int dev = 0, khz = 0;
        NNP_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            sv->tick_hz = double(khz) * 1e3;
        NNP_HIP(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&sv->arena), hbm_budget_bytes);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(sv->stream);
            set_error(std::string("could not reserve the HBM budget: ") + hipGetErrorString(e));
            return NNP_ENOMEM;
        }
        {
            Arena a(sv->arena, hbm_budget_bytes);
            carve_fixed(*sv, sv->n_cap, a);
        }
        if (hipHostMalloc(reinterpret_cast<void**>(&sv->stamps_host), sizeof(uint64_t) * (kMaxStepsPerCall + 1),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sv->repack_host), sizeof(RepackEntry) * max_slots,
                          hipHostMallocDefault) != hipSuccess) {
            if (sv->stamps_host) (void)hipHostFree(sv->stamps_host);
            (void)hipFree(sv->arena);
            (void)hipStreamDestroy(sv->stream);
            set_error("could not allocate pinned host memory");
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
    if (sv->stamps_host) (void)hipHostFree(sv->stamps_host);
    if (sv->repack_host) (void)hipHostFree(sv->repack_host);
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
        Dynamic D;
        // its lists and scratch, and its share of the fixed per-atom banks
        *bytes = carve_dynamic(sv, {&r}, nullptr, D) - sv.fixed_bytes +
                 size_t(double(sv.fixed_bytes) * double(n) / double(sv.n_cap));
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
        NNP_REQUIRE(fits(sv, {r.get()}), NNP_ENOMEM, "replica alone exceeds the HBM budget");
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
        for (int it = 0; it < max_outer_steps;) {
            boundary(sv);
            if (sv.resident.empty()) break;
            const int R = int(sv.resident.size());
            // advance to the next boundary at which a replica retires, within
            // the caller's step count
            int k = std::min(max_outer_steps - it, kMaxStepsPerCall);
            for (Replica* r : sv.resident) k = std::min(k, r->n_outer - r->steps_done);
            k = std::max(k, 1);
            std::vector<uint64_t> seeds(R), streams(R), base(R);
            std::vector<int> bad(R, 0);
            for (int j = 0; j < R; ++j) {
                seeds[j] = sv.resident[j]->seed;
                streams[j] = sv.resident[j]->stream_id;
                base[j] = sv.resident[j]->step;
            }
            respa_params p = sv.p;
            p.check_every = k;
            nnp_status e = respa_run(sv.cons, sv.nc, &sv.st, &p, k, sv.ws, sv.ws_bytes, sv.stream, seeds.data(),
                                     streams.data(), base.data(), bad.data(), sv.stamps);
            if (e == NNP_ECAPACITY) {
                grow_lists(sv);  // the state is back at the start of the call
                continue;
            }
            if (e != NNP_OK) return e;
            NNP_HIP(hipMemcpyAsync(sv.stamps_host, sv.stamps, sizeof(uint64_t) * k, hipMemcpyDeviceToHost,
                                   sv.stream));
            NNP_HIP(hipStreamSynchronize(sv.stream));
            for (int j = 0; j < R; ++j) {
                Replica* r = sv.resident[j];
                if (r->state == NNP_REPLICA_FAILED) continue;
                if (bad[j]) {
                    r->state = NNP_REPLICA_FAILED;
                    r->error = NNP_EUNSTABLE;
                    continue;
                }
                uint64_t prev = r->tick_last;
                for (int q = 0; q < k; ++q) {
                    sv.latencies.push_back(double(int64_t(sv.stamps_host[q] - prev)) / sv.tick_hz);
                    prev = sv.stamps_host[q];
                }
                r->tick_last = prev;
                r->steps_done += k;
                r->step += uint64_t(k) * uint64_t(sv.p.n_inner);
            }
            it += k;
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
