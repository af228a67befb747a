// Periodic cell-list neighbour build (gfx950).
//
// Pipeline for a packed multi-replica system (one launch each, every kernel
// a no-op when the device flag `run` is zero, so a rebuild can be decided on
// the device without a host round trip):
//   cell_assign  atom -> cell (per-replica grid of m^3 cells of edge >= rc,
//                numbered in the Morton order of their coordinates, or a
//                single cell holding the whole replica when m < 3),
//                counting-sort slot by atomic increment, and a copy of the
//                positions as the reference for the displacement trigger
//   scan         exclusive prefix sums of the cell counts
//   cell_fill    cell-sorted atom array
//   nbr_count    one wavefront per atom: 27-cell stencil, float64 pair rule
//   scan         row offsets
//   nbr_fill     same tests, ballot compaction into LDS, rank sort so each
//                row lists j ascending, then a coalesced row store
//   nbr_reverse  rev[e] for e = (i, j): position of i in row j (binary search)
// A second list at a smaller radius is filtered from the first row by row
// (filter_count / scan / filter_fill), which keeps row order.
//
// In cell order (the working order of the force evaluations inside the
// integrator) row p belongs to the atom at position p of the cell-sorted
// array and an entry names its neighbour by that position too; rows still
// list the neighbours in ascending caller index, so each atom's sums keep
// their order.  commit_order then records the permutation with the
// positions and species in that order, once both lists are built.
#include <algorithm>
#include <utility>

#include "common.h"
#include "kernels.h"
#include "model.h"

namespace nnp {

constexpr int kWaves = 4;          // wavefronts per block for per-atom kernels
constexpr int kMaxRow = 1024;      // longest row the fill kernels can sort

__global__ void k_set_flag(int* flag, int value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = value;
}

__global__ void k_cell_assign(int n, const double* __restrict__ pos, RepGeom geom,
                              const int* __restrict__ grid_m, const int* __restrict__ grid_base,
                              const int* __restrict__ cell_code,
                              const int* __restrict__ run, int* __restrict__ cell_of_atom,
                              int* __restrict__ slot_of_atom, int* __restrict__ cell_count,
                              double* __restrict__ pos_ref) {
    if (*run == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = geom.rep_of_atom ? geom.rep_of_atom[i] : 0;
    double L, inv;
    geom.get(i, L, inv);
    int m = grid_m[r];
    double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    if (pos_ref) {
        pos_ref[i] = x;
        pos_ref[n + i] = y;
        pos_ref[2 * n + i] = z;
    }
    int cell = grid_base[r];
    if (m > 1) {
        int c[3];
        double p[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double w = p[a] - L * floor(p[a] * inv);
            int ci = int(w * inv * double(m));
            c[a] = ci < 0 ? 0 : (ci >= m ? m - 1 : ci);
        }
        cell = cell_code[cell + (c[0] * m + c[1]) * m + c[2]];
    }
    cell_of_atom[i] = cell;
    slot_of_atom[i] = atomicAdd(&cell_count[cell], 1);
}

// Exclusive scan of in[0..n) into out[0..n] (out[n] = total), one block.
// Tiles of 1024 x 16 elements pass through LDS so that the global loads and
// stores are coalesced (element q * 1024 + t of the tile by thread t); in
// LDS thread t owns 16 consecutive elements: wavefront prefix sums of the
// thread totals, then the 16 wavefront totals; a carry links the tiles.
__global__ void __launch_bounds__(1024) k_scan(int n, const int* __restrict__ in,
                                                int* __restrict__ out, const int* __restrict__ run) {
    if (run && *run == 0) return;
    constexpr int E = 16, TILE = 1024 * E;
    __shared__ int tile[TILE + TILE / 32];  // one padding word per 32 (thread rows of 16 words)
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    auto at = [](int k) { return k + (k >> 5); };
    int carry = 0;
    for (int base = 0; base < n; base += TILE) {
        int g[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = base + q * 1024 + t;
            g[q] = k < n ? in[min(k, n - 1)] : 0;
        }
#pragma unroll
        for (int q = 0; q < E; ++q) tile[at(q * 1024 + t)] = g[q];
        __syncthreads();
        int v[E];
        int tot = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            v[k] = tile[at(t * E + k)];
            tot += v[k];
        }
        int inc = tot;  // inclusive prefix of the thread totals within the wavefront
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int before = carry, all = carry;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int x = wsum[q];
            if (q < w) before += x;
            all += x;
        }
        int run_sum = before + inc - tot;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            tile[at(t * E + k)] = run_sum;
            run_sum += v[k];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = base + q * 1024 + t;
            if (k < n) out[k] = tile[at(q * 1024 + t)];
        }
        carry = all;
        __syncthreads();  // tile and wsum are rewritten by the next tile
    }
    if (t == 0) out[n] = carry;
}

// Cell members in cell order, with a copy of their positions in the same
// order (SoA [3][n]): the candidates of a cell are then read contiguously.
__global__ void k_cell_fill(int n, const int* __restrict__ run, const int* __restrict__ cell_of_atom,
                            const int* __restrict__ slot_of_atom, const int* __restrict__ cell_start,
                            int* __restrict__ cell_atoms, const double* __restrict__ pos,
                            double* __restrict__ cell_pos) {
    if (*run == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = cell_start[cell_of_atom[i]] + slot_of_atom[i];
    cell_atoms[t] = i;
    cell_pos[t] = pos[i];
    cell_pos[n + t] = pos[n + i];
    cell_pos[2 * n + t] = pos[2 * n + i];
}

// Iterates over the stencil cells of atom i; calls body(t) for every
// candidate, t its position in cell order (-1: none for this lane).  With a cell grid the 27 cells' member lists are taken as one
// stream: lane k < 27 holds cell k's range, a wavefront prefix sum numbers
// the candidates, and each lane finds the cell of its candidate by a binary
// search over the lanes (every lane busy, about (27 x members) / 64 trips
// instead of 27).  Every candidate is visited once; the order does not
// matter to the callers (counts; rows sorted by j).
struct Stencil {
    const int* grid_m;
    const int* grid_base;
    const int* cell_code;  // lexicographic position -> cell number (CellPlan)
    const int* cell_lex;   // and back
    const int* cell_of_atom;
    const int* cell_start;
    const int* cell_atoms;
    const double* cell_pos;  // [3][n] positions in cell order
};

template <class Body>
__device__ __forceinline__ void for_candidates(const Stencil& st, int i, int r, int lane, Body body) {
    int m = st.grid_m[r];
    int base = st.grid_base[r];
    int cell = st.cell_of_atom[i];
    if (m == 1) {
        const int s = st.cell_start[cell], e = st.cell_start[cell + 1];
        const int trips = (e - s + 63) / 64;  // uniform across the wavefront
        for (int k = 0; k < trips; ++k) {
            const int t = s + k * 64 + lane;
            body(t < e ? t : -1);
        }
        return;
    }
    const int local = st.cell_lex[cell] - base;
    const int cx = local / (m * m), cy = (local / m) % m, cz = local % m;
    int start = 0, count = 0;
    if (lane < 27) {
        const int dx = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dz = lane % 3 - 1;
        const int ax = (cx + dx + m) % m, ay = (cy + dy + m) % m, az = (cz + dz + m) % m;
        const int c = st.cell_code[base + (ax * m + ay) * m + az];
        start = st.cell_start[c];
        count = st.cell_start[c + 1] - start;
    }
    int incl = count;  // inclusive prefix sum over lanes 0..26
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const int excl = incl - count;
    const int delta = start - excl;  // list position of candidate t of this cell: t + delta
    const int total = __shfl(incl, 26, 64);
    for (int t0 = 0; t0 < total; t0 += 64) {
        const int t = t0 + lane;
        // the largest cell k with excl_k <= t (empty cells are passed over)
        int k = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1) {
            const int cand = k + step;
            const int e = __shfl(excl, min(cand, 26), 64);
            if (cand <= 26 && e <= t) k = cand;
        }
        const int d = __shfl(delta, k, 64);
        body(t < total ? t + d : -1);
    }
}

// cell_rows: row p is the atom at cell position p (else row i is atom i)
__global__ void __launch_bounds__(64 * kWaves)
k_nbr_count(int n, const double* __restrict__ pos, RepGeom geom, Stencil st, double rc2,
            const int* __restrict__ run, int* __restrict__ counts, int* __restrict__ status, int cell_rows) {
    if (*run == 0) return;
    int lane = threadIdx.x & 63;
    const int row_i = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (row_i >= n) return;  // whole wavefront exits together
    const int i = cell_rows ? st.cell_atoms[row_i] : row_i;
    int r = geom.rep_of_atom ? geom.rep_of_atom[i] : 0;
    double L, inv;
    geom.get(i, L, inv);
    double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int cnt = 0;
    for_candidates(st, i, r, lane, [&](int t) {
        const int j = t >= 0 ? st.cell_atoms[t] : -1;
        if (j >= 0 && j != i) {
            double dx, dy, dz;
            if (pair_rule(xi, yi, zi, st.cell_pos[t], st.cell_pos[n + t], st.cell_pos[2 * n + t], L, inv, rc2, dx,
                          dy, dz))
                ++cnt;
        }
    });
    float tot = wave_sum(float(cnt));
    if (lane == 0) {
        const int c = int(tot + 0.5f);
        counts[row_i] = c;
        if (c > kMaxRow) status[2] = 1;  // the fill kernel cannot sort this row: build nothing
    }
}

// Rank sort of `cnt` distinct keys in LDS key[] into out[] (global): the
// entry of rank k is val[t] of the key of rank k (val = nullptr: the key).
__device__ __forceinline__ void rank_sort_store(const int* key, const int* val, int cnt, int lane, int* out) {
    for (int t = lane; t < cnt; t += 64) {
        int v = key[t];
        int rank = 0;
        for (int u = 0; u < cnt; ++u) rank += key[u] < v;
        out[rank] = val ? val[t] : v;
    }
}

__global__ void __launch_bounds__(64 * kWaves)
k_nbr_fill(int n, const double* __restrict__ pos, RepGeom geom, Stencil st, double rc2,
           const int* __restrict__ run, const int* __restrict__ tmp_off, int64_t capacity,
           int* __restrict__ offsets, int* __restrict__ nbr, int* __restrict__ status, int cell_rows) {
    if (*run == 0) return;
    __shared__ int rows[kWaves][kMaxRow];
    __shared__ int cpos[kWaves][kMaxRow];  // cell positions of the entries (cell_rows)
    int lane = threadIdx.x & 63;
    int w = threadIdx.x >> 6;
    const int row_i = xcd_block(blockIdx.x, gridDim.x) * kWaves + w;
    if (row_i >= n) return;
    const int i = cell_rows ? st.cell_atoms[row_i] : row_i;
    int total = tmp_off[n];
    if (status[2] != 0) return;  // a row is longer than kMaxRow: keep the previous list intact
    if (int64_t(total) > capacity) {
        if (i == 0 && lane == 0) {
            status[0] = 1;      // capacity overflow
            status[1] = total;  // required entries
        }
        return;
    }
    int r = geom.rep_of_atom ? geom.rep_of_atom[i] : 0;
    double L, inv;
    geom.get(i, L, inv);
    double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int fill = 0;
    int* row = rows[w];
    int* crow = cpos[w];
    for_candidates(st, i, r, lane, [&](int t) {
        const int j = t >= 0 ? st.cell_atoms[t] : -1;
        bool ok = false;
        if (j >= 0 && j != i) {
            double dx, dy, dz;
            ok = pair_rule(xi, yi, zi, st.cell_pos[t], st.cell_pos[n + t], st.cell_pos[2 * n + t], L, inv, rc2, dx,
                           dy, dz);
        }
        uint64_t bal = __ballot(ok);
        int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (ok && fill + pre < kMaxRow) {
            row[fill + pre] = j;
            crow[fill + pre] = t;
        }
        fill += __popcll(bal);
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    int start = tmp_off[row_i];
    if (fill != tmp_off[row_i + 1] - start) {
        if (lane == 0) status[3] = 1;  // count and fill disagree (not expected)
    }
    fill = min(fill, tmp_off[row_i + 1] - start);
    if (lane == 0) {
        offsets[row_i] = start;
        if (row_i == n - 1) offsets[n] = total;
    }
    // ascending caller index; stored as cell positions in cell order
    rank_sort_store(row, cell_rows ? crow : nullptr, fill, lane, nbr + start);
}

// Second list at a smaller radius, filtered from a first list row by row.
__global__ void __launch_bounds__(64 * kWaves)
k_filter_count(int n, const double* __restrict__ pos, RepGeom geom, const int* __restrict__ off_in,
               const int* __restrict__ nbr_in, double rc2, const int* __restrict__ run,
               int* __restrict__ counts, const int* __restrict__ src_status) {
    if (*run == 0 || (src_status && (src_status[0] | src_status[2]) != 0)) return;
    int lane = threadIdx.x & 63;
    int i = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (i >= n) return;
    double L, inv;
    geom.get(i, L, inv);
    double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int cnt = 0;
    for (int e = off_in[i] + lane; e < off_in[i + 1]; e += 64) {
        int j = nbr_in[e];
        double dx, dy, dz;
        cnt += pair_rule(xi, yi, zi, pos[j], pos[n + j], pos[2 * n + j], L, inv, rc2, dx, dy, dz);
    }
    float tot = wave_sum(float(cnt));
    if (lane == 0) counts[i] = int(tot + 0.5f);
}

__global__ void __launch_bounds__(64 * kWaves)
k_filter_fill(int n, const double* __restrict__ pos, RepGeom geom, const int* __restrict__ off_in,
              const int* __restrict__ nbr_in, double rc2, const int* __restrict__ run,
              const int* __restrict__ tmp_off, int64_t capacity, int* __restrict__ offsets,
              int* __restrict__ nbr, int* __restrict__ status, const int* __restrict__ src_status) {
    if (*run == 0 || (src_status && (src_status[0] | src_status[2]) != 0)) return;
    int lane = threadIdx.x & 63;
    int i = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (i >= n) return;
    int total = tmp_off[n];
    if (int64_t(total) > capacity) {
        if (i == 0 && lane == 0) {
            status[0] = 1;
            status[1] = total;
        }
        return;
    }
    double L, inv;
    geom.get(i, L, inv);
    double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int out = tmp_off[i];
    int s = off_in[i], e_end = off_in[i + 1];
    for (int base = s; base < e_end; base += 64) {
        int e = base + lane;
        bool ok = false;
        int j = -1;
        if (e < e_end) {
            j = nbr_in[e];
            double dx, dy, dz;
            ok = pair_rule(xi, yi, zi, pos[j], pos[n + j], pos[2 * n + j], L, inv, rc2, dx, dy, dz);
        }
        uint64_t bal = __ballot(ok);
        int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (ok) nbr[out + pre] = j;
        out += __popcll(bal);
    }
    if (lane == 0) {
        offsets[i] = tmp_off[i];
        if (i == n - 1) offsets[n] = total;
    }
}

// key (or nullptr): the caller's index of a row (rows in cell order list
// their entries in ascending key)
__global__ void __launch_bounds__(64 * kWaves)
k_nbr_reverse(int n, const int* __restrict__ run, const int* __restrict__ status,
              const int* __restrict__ offsets, const int* __restrict__ nbr, int* __restrict__ rev,
              const int* __restrict__ key) {
    if (*run == 0 || status[0] != 0 || status[2] != 0) return;
    int lane = threadIdx.x & 63;
    int i = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (i >= n) return;
    const int ki = key ? key[i] : i;
    for (int e = offsets[i] + lane; e < offsets[i + 1]; e += 64) {
        int j = nbr[e];
        int lo = offsets[j], hi = offsets[j + 1];  // search i in row j (ascending key)
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if ((key ? key[nbr[mid]] : nbr[mid]) < ki) lo = mid + 1; else hi = mid;
        }
        rev[e] = (lo < offsets[j + 1] && nbr[lo] == i) ? lo : e;
    }
}

// After a successful build in cell order: order[p] = caller's index of row
// p, order[n + i] = row of atom i, and the positions and species in row
// order for the evaluations (a failed build keeps the previous order with
// the previous lists).
__global__ void k_commit_order(int n, const int* __restrict__ run, const int* __restrict__ status,
                               const int* __restrict__ cell_atoms, const double* __restrict__ cell_pos,
                               const int* __restrict__ species, int* __restrict__ order, double* __restrict__ pos_m,
                               int* __restrict__ species_m) {
    if (*run == 0 || status[0] != 0 || status[2] != 0) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = cell_atoms[p];
    order[p] = i;
    order[n + i] = p;
    pos_m[p] = cell_pos[p];
    pos_m[n + p] = cell_pos[n + p];
    pos_m[2 * n + p] = cell_pos[2 * n + p];
    species_m[p] = species[i];
}

// A list built into spare buffers (with its order and row-ordered copies)
// replaces the one in use, once nothing reads the latter any more; only
// after a build that ran and succeeded.
__global__ void k_adopt_lists(int n, const int* __restrict__ run, const int* __restrict__ status,
                              const int* __restrict__ off_src, const int* __restrict__ nbr_src, int64_t capacity,
                              int* __restrict__ off_dst, int* __restrict__ nbr_dst, const int* __restrict__ order_src,
                              int* __restrict__ order_dst, const double* __restrict__ pos_src,
                              double* __restrict__ pos_dst, const int* __restrict__ sp_src, int* __restrict__ sp_dst) {
    if (*run == 0 || status[0] != 0 || status[2] != 0) return;
    const int64_t total = min(int64_t(off_src[n]), capacity);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) nbr_dst[t] = nbr_src[t];
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t <= n; t += stride) {
        off_dst[t] = off_src[t];
        if (t < n && order_src) {
            order_dst[t] = order_src[t];
            order_dst[n + t] = order_src[n + t];
            pos_dst[t] = pos_src[t];
            pos_dst[n + t] = pos_src[n + t];
            pos_dst[2 * n + t] = pos_src[2 * n + t];
            sp_dst[t] = sp_src[t];
        }
    }
}

// Positions and species in row order from the caller's arrays (order ==
// nullptr: the identity, also written to `reset`).  Indices read from
// `order` are clamped to [0, n): a buffer that no build has written yet
// still leads to no access out of bounds.
__global__ void k_gather_rows(int n, const int* __restrict__ order, const double* __restrict__ pos,
                              const int* __restrict__ species, double* __restrict__ pos_m,
                              int* __restrict__ species_m, int* __restrict__ reset) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = order ? min(max(order[p], 0), n - 1) : p;
    if (reset) {
        reset[p] = p;
        reset[n + p] = p;
    }
    pos_m[p] = pos[i];
    pos_m[n + p] = pos[n + i];
    pos_m[2 * n + p] = pos[2 * n + i];
    if (species_m) species_m[p] = species[i];
}

__global__ void k_disp_check(int n, const double* __restrict__ pos, const double* __restrict__ ref,
                             double thr2, int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool over = false;
    if (i < n) {
        double dx = pos[i] - ref[i], dy = pos[n + i] - ref[n + i], dz = pos[2 * n + i] - ref[2 * n + i];
        double d2 = dx * dx + dy * dy + dz * dz;
        over = !(d2 <= thr2);  // NaN also triggers
    }
    if (__ballot(over) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void k_finish_rebuild(int* flag, long long* n_rebuilds, unsigned* maxd2) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (*flag) {
            if (n_rebuilds) *n_rebuilds += 1;
            if (maxd2) {
                maxd2[0] = 0u;
                maxd2[1] = 0u;
            }
            *flag = 0;
        }
    }
}

// maxd2 holds non-negative floats as bits (their order is that of the
// unsigned integers).  Growth over the last outer step is extrapolated
// twice over; the hard per-step check in k_baoa guards the rest.
__global__ void k_predict_rebuild(unsigned* maxd2, double thr, int* flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double d = sqrt(double(__uint_as_float(maxd2[0])));
        const double dp = sqrt(double(__uint_as_float(maxd2[1])));
        const double pred = d + 2.0 * fmax(d - dp, 0.0);
        if (!(pred < thr)) *flag = 1;  // also for non-finite displacements
        maxd2[1] = maxd2[0];
    }
}

// ------------------------------------------------------------------- host --

// Morton rank of each lexicographic cell position of an m^3 grid: the cells
// sorted by their bit-interleaved coordinates (x, y, z bits in turn).
static std::vector<int> morton_ranks(int m) {
    const int n = m * m * m;
    std::vector<std::pair<uint64_t, int>> key(n);
    for (int l = 0; l < n; ++l) {
        const int c[3] = {l / (m * m), (l / m) % m, l % m};
        uint64_t code = 0;
        for (int b = 0; b < 20; ++b)
            for (int d = 0; d < 3; ++d) code |= uint64_t((c[d] >> b) & 1) << (3 * b + (2 - d));
        key[l] = {code, l};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> rank(n);
    for (int k = 0; k < n; ++k) rank[key[k].second] = k;
    return rank;
}

CellPlan plan_cells(const nnp_system& sys, double radius) {
    CellPlan p;
    p.m.resize(sys.n_rep);
    p.base.resize(sys.n_rep);
    int total = 0;
    for (int r = 0; r < sys.n_rep; ++r) {
        double L = sys.box[r];
        NNP_REQUIRE(L > 0 && radius < 0.5 * L, NNP_EINVAL,
                    "pair radius must be below half the box edge (replica " + std::to_string(r) + ")");
        int64_t nr = sys.rep_start[r + 1] - sys.rep_start[r];
        int m = int(std::floor(L / (radius * (1.0 + 1e-9))));
        while (m >= 3 && int64_t(m) * m * m > 2 * nr + 27) --m;
        if (m < 3) m = 1;
        p.m[r] = m;
        p.base[r] = total;
        total += m * m * m;
    }
    p.n_cells = total;
    p.code.resize(total);
    p.lex.resize(total);
    std::vector<int> rank;
    int rank_m = 0;
    for (int r = 0; r < sys.n_rep; ++r) {
        const int m = p.m[r], b = p.base[r], nc = m * m * m;
        if (m != rank_m) {
            rank = morton_ranks(m);
            rank_m = m;
        }
        for (int l = 0; l < nc; ++l) {
            p.code[b + l] = b + rank[l];
            p.lex[b + rank[l]] = b + l;
        }
    }
    return p;
}

int64_t max_cells(int64_t n_atoms, int32_t n_rep) { return 2 * n_atoms + 27 * int64_t(n_rep) + 1; }

void carve_nbr_scratch(Arena& a, int64_t n, int32_t n_rep, NbrScratch& s) {
    int64_t C = max_cells(n, n_rep);
    s.grid_m = a.take<int>(n_rep);
    s.grid_base = a.take<int>(n_rep);
    s.cell_code = a.take<int>(C + 1);
    s.cell_lex = a.take<int>(C + 1);
    s.cell_of_atom = a.take<int>(n);
    s.slot_of_atom = a.take<int>(n);
    s.cell_count = a.take<int>(C + 1);
    s.cell_start = a.take<int>(C + 1);
    s.cell_atoms = a.take<int>(n);
    s.cell_pos = a.take<double>(3 * n);
    s.counts = a.take<int>(n);
    s.tmp_off = a.take<int>(n + 1);
    s.status = a.take<int>(8);
}

void upload_cell_plan(const CellPlan& plan, NbrScratch& s, hipStream_t stream) {
    NNP_HIP(hipMemcpyAsync(s.cell_code, plan.code.data(), plan.code.size() * sizeof(int), hipMemcpyHostToDevice,
                           stream));
    NNP_HIP(hipMemcpyAsync(s.cell_lex, plan.lex.data(), plan.lex.size() * sizeof(int), hipMemcpyHostToDevice,
                           stream));
    NNP_HIP(hipMemcpyAsync(s.grid_m, plan.m.data(), plan.m.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    NNP_HIP(hipMemcpyAsync(s.grid_base, plan.base.data(), plan.base.size() * sizeof(int),
                           hipMemcpyHostToDevice, stream));
}

void launch_build(int n, const double* pos, const RepGeom& geom, const CellPlan& plan, NbrScratch& s,
                  const int* run, double radius, int64_t capacity, int* offsets, int* nbr, int* rev,
                  double* pos_ref, hipStream_t stream, bool cell_rows) {
    launch_zero(s.cell_count, plan.n_cells + 1, run, stream);
    k_cell_assign<<<cdiv(n, 256), 256, 0, stream>>>(n, pos, geom, s.grid_m, s.grid_base, s.cell_code, run,
                                                    s.cell_of_atom, s.slot_of_atom, s.cell_count, pos_ref);
    k_scan<<<1, 1024, 0, stream>>>(plan.n_cells, s.cell_count, s.cell_start, run);
    k_cell_fill<<<cdiv(n, 256), 256, 0, stream>>>(n, run, s.cell_of_atom, s.slot_of_atom, s.cell_start,
                                                  s.cell_atoms, pos, s.cell_pos);
    Stencil st{s.grid_m, s.grid_base, s.cell_code, s.cell_lex, s.cell_of_atom, s.cell_start, s.cell_atoms, s.cell_pos};
    double rc2 = radius * radius;
    const int cr = cell_rows ? 1 : 0;
    k_nbr_count<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, pos, geom, st, rc2, run, s.counts, s.status, cr);
    k_scan<<<1, 1024, 0, stream>>>(n, s.counts, s.tmp_off, run);
    ScopedTimer timer("nbr_fill", stream);
    k_nbr_fill<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, pos, geom, st, rc2, run, s.tmp_off, capacity,
                                                            offsets, nbr, s.status, cr);
    if (rev)
        k_nbr_reverse<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, run, s.status, offsets, nbr, rev,
                                                                   cell_rows ? s.cell_atoms : nullptr);
    NNP_LAUNCH_CHECK();
}

void launch_commit_order(int n, const NbrScratch& s, const int* run, const int* species, int* order,
                         double* pos_m, int* species_m, hipStream_t stream) {
    k_commit_order<<<cdiv(n, 256), 256, 0, stream>>>(n, run, s.status, s.cell_atoms, s.cell_pos, species, order,
                                                     pos_m, species_m);
    NNP_LAUNCH_CHECK();
}

void launch_gather_rows(int n, const int* order, const double* pos, const int* species, double* pos_m,
                        int* species_m, hipStream_t stream) {
    if (n <= 0) return;
    k_gather_rows<<<cdiv(n, 256), 256, 0, stream>>>(n, order, pos, species, pos_m, species_m, nullptr);
    NNP_LAUNCH_CHECK();
}

void launch_adopt_lists(int n, const int* run, const NbrScratch& s, const int* off_src, const int* nbr_src,
                        int64_t capacity, int* off_dst, int* nbr_dst, const int* order_src, int* order_dst,
                        const double* pos_src, double* pos_dst, const int* sp_src, int* sp_dst, hipStream_t stream) {
    if (n <= 0) return;
    k_adopt_lists<<<1024, 256, 0, stream>>>(n, run, s.status, off_src, nbr_src, capacity, off_dst, nbr_dst, order_src,
                                            order_dst, pos_src, pos_dst, sp_src, sp_dst);
    NNP_LAUNCH_CHECK();
}

void launch_reset_rows(int n, int* order, const double* pos, const int* species, double* pos_m, int* species_m,
                       hipStream_t stream) {
    if (n <= 0) return;
    k_gather_rows<<<cdiv(n, 256), 256, 0, stream>>>(n, nullptr, pos, species, pos_m, species_m, order);
    NNP_LAUNCH_CHECK();
}

void launch_filter(int n, const double* pos, const RepGeom& geom, NbrScratch& s, const int* run,
                   const int* off_in, const int* nbr_in, double radius, int64_t capacity, int* offsets,
                   int* nbr, int* rev, int* status, hipStream_t stream, const int* key, const int* src_status) {
    double rc2 = radius * radius;
    k_filter_count<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, pos, geom, off_in, nbr_in, rc2, run, s.counts,
                                                                src_status);
    k_scan<<<1, 1024, 0, stream>>>(n, s.counts, s.tmp_off, run);
    k_filter_fill<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, pos, geom, off_in, nbr_in, rc2, run, s.tmp_off,
                                                               capacity, offsets, nbr, status, src_status);
    if (rev)
        k_nbr_reverse<<<cdiv(n, kWaves), 64 * kWaves, 0, stream>>>(n, run, status, offsets, nbr, rev, key);
    NNP_LAUNCH_CHECK();
}

void launch_set_flag(int* flag, int value, hipStream_t stream) {
    k_set_flag<<<1, 64, 0, stream>>>(flag, value);
    NNP_LAUNCH_CHECK();
}

void launch_disp_check(int n, const double* pos, const double* ref, double thr, int* flag, hipStream_t stream) {
    k_disp_check<<<cdiv(n, 256), 256, 0, stream>>>(n, pos, ref, thr * thr, flag);
    NNP_LAUNCH_CHECK();
}

void launch_finish_rebuild(int* flag, long long* n_rebuilds, unsigned* maxd2, hipStream_t stream) {
    k_finish_rebuild<<<1, 64, 0, stream>>>(flag, n_rebuilds, maxd2);
    NNP_LAUNCH_CHECK();
}

void launch_predict_rebuild(unsigned* maxd2, double thr, int* flag, hipStream_t stream) {
    k_predict_rebuild<<<1, 64, 0, stream>>>(maxd2, thr, flag);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp

namespace nnp {
void launch_reverse(int n, const int* run, const int* status, const int* offsets, const int* nbr, int* rev,
                    hipStream_t s) {
    k_nbr_reverse<<<cdiv(n, kWaves), 64 * kWaves, 0, s>>>(n, run, status, offsets, nbr, rev, nullptr);
    NNP_LAUNCH_CHECK();
}
}  // namespace nnp
