// kernels.hip -- the per-step kernels of the molecule-agent update for
// gfx950 (wave64).  One step (O2..O10 of the step definition) is
//
//   move      unimolecular draw, Brownian move, boundaries, event effects,
//             cell key + rank by per-cell atomic count, birth records
//   scan      exclusive prefix sum of the cell counts (reduce, top, down)
//   scatter   agents to cell-sorted order in the other buffer, holes and
//             degraded agents dropped (stream compaction)
//   propose   nearest eligible partner of each claimer over the cell
//             stencil, Bernoulli draw, handshake keys into the claim slots
//   apply     confirmed pairs fire
//   births    children sorted by parent id, appended with fresh ids; step
//             bookkeeping
//
// All agent data are structure-of-arrays, one thread per agent, so every
// streaming access is coalesced.  No kernel here is a dense contraction.
#include "device_math.hpp"
#include "engine.hpp"

namespace mabm {

const char* const kKernelNames[kNumKernels] = {"move", "scan_reduce", "scan_top", "scan_down",
                                               "scatter", "propose", "apply", "births"};

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t grid_blocks_for(uint32_t n) { return (n + kBlock - 1) / kBlock; }

// ---------------------------------------------------------------------------
// O0: initial placement.  Agent i (id i) belongs to the first species whose
// prefix end exceeds i; attempt a uses INIT(i, a) and keeps the first
// uniform point of its compartment's bounding box inside that compartment.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_init(Dev d)
{
    const Tables& T = *d.tab;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.n_init) return;
    int s = 0;
    while (s < T.ns - 1 && i >= T.init_end[s]) ++s;
    const int c = T.init_comp[s];
    float x = 0.0f, y = 0.0f, z = 0.0f;
    bool ok = false;
    for (uint32_t a = 0; a < 64u && !ok; ++a) {
        const U4 w = draw(T, i, a, kInit, 0u);
        if (T.geometry == kBox) {
            x = wrap_box(T, u01(w.w0) * T.L);
            y = wrap_box(T, u01(w.w1) * T.L);
            z = wrap_box(T, u01(w.w2) * T.L);
            ok = true;
        } else {
            const float R = (T.geometry == kNested && c == 0) ? T.Rin : T.Rout;
            x = (u01(w.w0) * 2.0f - 1.0f) * R;
            y = (u01(w.w1) * 2.0f - 1.0f) * R;
            z = (u01(w.w2) * 2.0f - 1.0f) * R;
            const float n2 = sq3(x, y, z);
            if (T.geometry == kSphere) ok = n2 <= T.Rout2;
            else if (c == 0) ok = n2 < T.Rin2;
            else ok = n2 >= T.Rin2 && n2 <= T.Rout2;
        }
    }
    if (!ok) atomicOr(&d.ctl->err, kErrPlacement);
    Agents A = d.a[0];
    A.x[i] = x;
    A.y[i] = y;
    A.z[i] = z;
    A.id[i] = i;
    A.sp[i] = uint8_t(s);
    d.rkey[i] = kNone;
    d.revent[i] = kNoEvent;
    d.rpartner[i] = kNone;
}

__global__ void __launch_bounds__(kBlock) k_fill_records(Dev d)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.capacity) return;
    d.rkey[i] = kNone;
    d.revent[i] = kNoEvent;
    d.rpartner[i] = kNone;
}

// Release offset of a split or emission (O8): cube rejection in the ball of
// radius `release`, BIRTH(id, t, attempt) for attempt < 8; every placed
// product must be admissible in the parent's compartment; else u = 0.
__device__ void release_offset(const Tables& T, const RuleDev& R, uint32_t id, uint32_t t,
                               float px, float py, float pz, bool both, float& ux, float& uy,
                               float& uz)
{
    const int c = compartment(T, px, py, pz);
    for (uint32_t a = 0; a < 8u; ++a) {
        const U4 w = draw(T, id, t, kBirth, a);
        const float vx = (u01(w.w0) * 2.0f - 1.0f) * R.release;
        const float vy = (u01(w.w1) * 2.0f - 1.0f) * R.release;
        const float vz = (u01(w.w2) * 2.0f - 1.0f) * R.release;
        if (!(sq3(vx, vy, vz) <= R.release2)) continue;
        float qx = px + vx, qy = py + vy, qz = pz + vz;
        if (T.geometry == kBox) {
            qx = wrap_box(T, qx);
            qy = wrap_box(T, qy);
            qz = wrap_box(T, qz);
        }
        if (!admissible(T, qx, qy, qz, c)) continue;
        if (both) {
            float rx = px - vx, ry = py - vy, rz = pz - vz;
            if (T.geometry == kBox) {
                rx = wrap_box(T, rx);
                ry = wrap_box(T, ry);
                rz = wrap_box(T, rz);
            }
            if (!admissible(T, rx, ry, rz, c)) continue;
        }
        ux = vx;
        uy = vy;
        uz = vz;
        return;
    }
    ux = uy = uz = 0.0f;
}

__device__ __forceinline__ void push_birth(const Dev& d, uint32_t parent, int sp, float x, float y,
                                           float z)
{
    const uint32_t k = atomicAdd(&d.ctl->n_births, 1u);
    if (k < kMaxBirthsPerStep) d.births[k] = Birth{parent, uint32_t(sp), x, y, z};
}

// ---------------------------------------------------------------------------
// move: O2 (event draw), O3 (Brownian step), O4 (boundaries), O5 and the
// unimolecular part of O8, then the cell key of the moved position and its
// rank within the cell (atomic count).  Final position and species are
// written back in place; busy agents are flagged.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_move(Dev d, int cur, int record)
{
    const Tables& T = *d.tab;
    Ctl* ctl = d.ctl;
    const uint32_t n = ctl->n_slots;
    const uint32_t t = ctl->t;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    __shared__ uint32_t live;
    if (threadIdx.x == 0) live = 0;
    __syncthreads();
    if (i < n) {
        Agents A = d.a[cur];
        const uint32_t s = A.sp[i];
        if (s == kDead) {
            d.key[i] = kNone;
        } else {
            atomicAdd(&live, 1u);
            const uint32_t id = A.id[i];
            const float x = A.x[i], y = A.y[i], z = A.z[i];
            const int c0 = compartment(T, x, y, z);

            int ev = -1;
            const int nu = T.uni_n[s][c0];
            if (nu) {
                const uint32_t w = draw(T, id, t, kUni, 0u).w0;
                for (int j = 0; j < nu; ++j)
                    if (uint64_t(w) < T.uni_thr[s][c0][j]) {
                        ev = T.uni_rule[s][c0][j];
                        break;
                    }
            }

            float z0, z1, z2;
            normals3(T, id, t, z0, z1, z2);
            const float sg = T.sigma[s];
            float x1 = x + sg * z0, y1 = y + sg * z1, w1 = z + sg * z2;
            if (T.geometry == kBox) {
                x1 = wrap_box(T, x1);
                y1 = wrap_box(T, y1);
                w1 = wrap_box(T, w1);
            } else {
                const float n2 = sq3(x1, y1, w1);
                bool reject = n2 > T.Rout2;
                if (T.geometry == kNested && !reject && (n2 < T.Rin2 ? 0 : 1) != c0) reject = true;
                if (reject) {
                    x1 = x;
                    y1 = y;
                    w1 = z;
                }
            }
            const uint32_t key = cell_of(T, x1, y1, w1);

            uint32_t fs = s;
            float fx = x1, fy = y1, fz = w1;
            bool dies = false;
            if (ev >= 0) {
                const RuleDev& R = T.rule[ev];
                float ux, uy, uz;
                switch (R.placement) {
                case kKeep:
                    if (R.p0 < 0) dies = true;
                    else fs = uint32_t(R.p0);
                    break;
                case kTranslocate: {
                    const float n2 = sq3(x1, y1, w1);
                    if (n2 == 0.0f) {
                        fx = R.target_r;
                        fy = 0.0f;
                        fz = 0.0f;
                    } else {
                        const float f = R.target_r / __builtin_sqrtf(n2);
                        fx = x1 * f;
                        fy = y1 * f;
                        fz = w1 * f;
                    }
                    if (R.p0 >= 0) fs = uint32_t(R.p0);
                    break;
                }
                case kSplit: {
                    release_offset(T, R, id, t, x1, y1, w1, true, ux, uy, uz);
                    fs = uint32_t(R.p0);
                    fx = x1 + ux;
                    fy = y1 + uy;
                    fz = w1 + uz;
                    float cx = x1 - ux, cy = y1 - uy, cz = w1 - uz;
                    if (T.geometry == kBox) {
                        fx = wrap_box(T, fx);
                        fy = wrap_box(T, fy);
                        fz = wrap_box(T, fz);
                        cx = wrap_box(T, cx);
                        cy = wrap_box(T, cy);
                        cz = wrap_box(T, cz);
                    }
                    push_birth(d, id, R.p1, cx, cy, cz);
                    break;
                }
                default: {  // kEmit
                    release_offset(T, R, id, t, x1, y1, w1, false, ux, uy, uz);
                    if (R.p0 >= 0) fs = uint32_t(R.p0);
                    float cx = x1 + ux, cy = y1 + uy, cz = w1 + uz;
                    if (T.geometry == kBox) {
                        cx = wrap_box(T, cx);
                        cy = wrap_box(T, cy);
                        cz = wrap_box(T, cz);
                    }
                    push_birth(d, id, R.p1, cx, cy, cz);
                    break;
                }
                }
            }
            if (dies) {
                d.key[i] = kNone;
            } else {
                A.x[i] = fx;
                A.y[i] = fy;
                A.z[i] = fz;
                A.sp[i] = uint8_t(fs);
                d.key[i] = key;
                d.rank[i] = atomicAdd(&d.cell_count[key], 1u);
                d.flag[i] = ev >= 0 ? 1 : 0;
                if (record) d.event[i] = ev >= 0 ? uint8_t(ev) : kNoEvent;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && live) atomicAdd(&ctl->agent_updates, (unsigned long long)live);
}

// ---------------------------------------------------------------------------
// scan of the cell counts: per-tile sums, one workgroup over the tile sums,
// per-tile exclusive scan with the tile offset (counts cleared for the next
// step).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan over a 256-thread block; returns the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < wv) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Dev d)
{
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < d.ncells) s += d.cell_count[base + k];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) d.tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(Dev d)
{
    uint32_t carry = 0;
    for (uint32_t b = 0; b < d.ntiles; b += kScanThreads) {
        const uint32_t k = b + threadIdx.x;
        const uint32_t v = k < d.ntiles ? d.tile_sum[k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (k < d.ntiles) d.tile_sum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        d.ctl->n_binned = carry;
        d.cell_start[d.ncells] = carry;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(Dev d)
{
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < d.ncells ? d.cell_count[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = d.tile_sum[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < d.ncells) {
            d.cell_start[base + k] = run;
            d.cell_count[base + k] = 0u;
        }
        run += v[k];
    }
}

// ---------------------------------------------------------------------------
// scatter: binned agents to cell order in the other buffer (O9 compaction
// of holes and degraded agents happens here: they carry no key).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_scatter(Dev d, int cur, int record)
{
    const uint32_t n = d.ctl->n_slots;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = d.key[i];
    if (key == kNone) return;
    const uint32_t j = d.cell_start[key] + d.rank[i];
    const Agents A = d.a[cur];
    const Agents B = d.a[cur ^ 1];
    B.x[j] = A.x[i];
    B.y[j] = A.y[i];
    B.z[j] = A.z[i];
    B.id[j] = A.id[i];
    B.sp[j] = A.sp[i];
    d.sflag[j] = d.flag[i];
    d.slot[j] = ~0ull;
    if (record) {
        d.rkey[j] = key;
        d.revent[j] = d.event[i];
        d.rpartner[j] = kNone;
    }
}

// ---------------------------------------------------------------------------
// propose (O7): for each non-busy claimer, the eligible partner minimising
// (d^2, id) over the 8-cell (h >= 2 R_max) or 27-cell stencil; a Bernoulli
// draw; both claim slots take the handshake key by atomic minimum.
// ---------------------------------------------------------------------------
struct Best {
    uint32_t idx, id;
    float d2;
    int rule;
};

__device__ __forceinline__ void scan_cell(const Dev& d, const Tables& T, const Agents& A,
                                          uint32_t cell, uint32_t self, uint32_t s, float x,
                                          float y, float z, int comp, Best& b)
{
    const uint32_t e = d.cell_start[cell + 1];
    for (uint32_t k = d.cell_start[cell]; k < e; ++k) {
        if (k == self) continue;
        const int r = T.rule_of[s][A.sp[k]];
        if (r < 0 || d.sflag[k]) continue;
        const float bx = A.x[k], by = A.y[k], bz = A.z[k];
        if (T.geometry == kNested && compartment(T, bx, by, bz) != comp) continue;
        float dx = bx - x, dy = by - y, dz = bz - z;
        if (T.geometry == kBox) {
            if (dx > T.halfL) dx -= T.L; else if (dx < -T.halfL) dx += T.L;
            if (dy > T.halfL) dy -= T.L; else if (dy < -T.halfL) dy += T.L;
            if (dz > T.halfL) dz -= T.L; else if (dz < -T.halfL) dz += T.L;
        }
        const float d2 = dx * dx + dy * dy + dz * dz;
        if (!(d2 <= T.rule[r].r2)) continue;
        const uint32_t bid = A.id[k];
        if (b.idx == kNone || d2 < b.d2 || (d2 == b.d2 && bid < b.id)) {
            b.idx = k;
            b.id = bid;
            b.d2 = d2;
            b.rule = r;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_propose(Dev d, int nxt)
{
    const Tables& T = *d.tab;
    const uint32_t n = d.ctl->n_binned;
    const uint32_t t = d.ctl->t;
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const Agents A = d.a[nxt];
    const uint32_t s = A.sp[j];
    uint32_t out = kNone;
    if (!d.sflag[j] && T.claimer[s]) {
        const float x = A.x[j], y = A.y[j], z = A.z[j];
        const int comp = compartment(T, x, y, z);
        const int G = int(T.G);
        int c[3], lo[3], hi[3], step[3];
        const float p[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            c[a] = int(cell_coord(T, p[a]));
            if (T.stencil8) {
                const float f = (p[a] - T.lo) * T.inv_h - float(c[a]);
                lo[a] = 0;
                hi[a] = 1;
                step[a] = f < 0.5f ? -1 : 1;
            } else {
                lo[a] = -1;
                hi[a] = 1;
                step[a] = 1;
            }
        }
        Best b{kNone, 0u, 0.0f, -1};
        const bool periodic = T.geometry == kBox;
        for (int oz = lo[2]; oz <= hi[2]; ++oz) {
            int cz = c[2] + oz * step[2];
            if (periodic) cz = (cz + G) % G; else if (cz < 0 || cz >= G) continue;
            for (int oy = lo[1]; oy <= hi[1]; ++oy) {
                int cy = c[1] + oy * step[1];
                if (periodic) cy = (cy + G) % G; else if (cy < 0 || cy >= G) continue;
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    int cx = c[0] + ox * step[0];
                    if (periodic) cx = (cx + G) % G; else if (cx < 0 || cx >= G) continue;
                    const uint32_t cell = uint32_t(cx) + T.G * (uint32_t(cy) + T.G * uint32_t(cz));
                    scan_cell(d, T, A, cell, j, s, x, y, z, comp, b);
                }
            }
        }
        if (b.idx != kNone) {
            const uint32_t ida = A.id[j];
            const uint32_t w = draw(T, ida, t, kPair, 0u).w0;
            if (uint64_t(w) < T.rule[b.rule].thr) {
                const uint32_t lo_id = ida < b.id ? ida : b.id, hi_id = ida < b.id ? b.id : ida;
                const unsigned long long pr =
                    (unsigned long long)draw(T, lo_id, t, kPrio, hi_id).w0 << 32;
                atomicMin(&d.slot[j], pr | b.id);
                atomicMin(&d.slot[b.idx], pr | ida);
                out = b.idx;
            }
        }
    }
    d.prop[j] = out;
}

// ---------------------------------------------------------------------------
// apply (O7 confirmation, O8 pair products).  Only the claimer of a
// confirmed pair writes, and of a mutual (homotypic) pair only the lower id.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_apply(Dev d, int nxt, int record)
{
    const Tables& T = *d.tab;
    const uint32_t n = d.ctl->n_binned;
    const uint32_t t = d.ctl->t;
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t b = d.prop[j];
    if (b == kNone) return;
    const Agents A = d.a[nxt];
    const uint32_t ida = A.id[j], idb = A.id[b];
    const uint32_t lo_id = ida < idb ? ida : idb, hi_id = ida < idb ? idb : ida;
    const unsigned long long pr = (unsigned long long)draw(T, lo_id, t, kPrio, hi_id).w0 << 32;
    if (d.slot[j] != (pr | idb) || d.slot[b] != (pr | ida)) return;
    if (d.prop[b] == j && idb < ida) return;
    const RuleDev& R = T.rule[T.rule_of[A.sp[j]][A.sp[b]]];
    A.sp[j] = R.p0 < 0 ? kDead : uint8_t(R.p0);
    A.sp[b] = R.p1 < 0 ? kDead : uint8_t(R.p1);
    if (record) {
        d.rpartner[j] = idb;
        d.rpartner[b] = ida;
    }
}

// ---------------------------------------------------------------------------
// births (O9, O10): one workgroup sorts this step's birth records by parent
// id (bitonic, in LDS), appends the children after the binned agents with
// ids next_id, next_id + 1, ..., and advances the step bookkeeping.
// ---------------------------------------------------------------------------
constexpr int kBirthThreads = 1024;

__global__ void __launch_bounds__(kBirthThreads) k_births(Dev d, int nxt, int record)
{
    __shared__ uint32_t skey[kMaxBirthsPerStep];
    __shared__ uint32_t sidx[kMaxBirthsPerStep];
    Ctl* ctl = d.ctl;
    const uint32_t nbin = ctl->n_binned;
    uint32_t nb = ctl->n_births;
    bool overflow = false;
    if (nb > kMaxBirthsPerStep) {
        overflow = true;
        nb = 0;
    } else if (uint64_t(nbin) + nb > d.capacity) {
        overflow = true;
        nb = 0;
    }
    if (nb > 0) {
        uint32_t np = 1;
        while (np < nb) np <<= 1;
        for (uint32_t k = threadIdx.x; k < np; k += kBirthThreads) {
            skey[k] = k < nb ? d.births[k].parent : 0xFFFFFFFFu;
            sidx[k] = k;
        }
        __syncthreads();
        for (uint32_t size = 2; size <= np; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t k = threadIdx.x; k < np; k += kBirthThreads) {
                    const uint32_t o = k ^ stride;
                    if (o > k) {
                        const bool up = (k & size) == 0;
                        const uint32_t a = skey[k], b = skey[o];
                        if ((a > b) == up) {
                            skey[k] = b;
                            skey[o] = a;
                            const uint32_t ti = sidx[k];
                            sidx[k] = sidx[o];
                            sidx[o] = ti;
                        }
                    }
                }
                __syncthreads();
            }
        }
        const Agents A = d.a[nxt];
        const uint32_t base_id = ctl->next_id;
        for (uint32_t r = threadIdx.x; r < nb; r += kBirthThreads) {
            const Birth bb = d.births[sidx[r]];
            const uint32_t j = nbin + r;
            A.x[j] = bb.x;
            A.y[j] = bb.y;
            A.z[j] = bb.z;
            A.id[j] = base_id + r;
            A.sp[j] = uint8_t(bb.sp);
            if (record) {
                d.rkey[j] = kNone;
                d.revent[j] = kNoEvent;
                d.rpartner[j] = kNone;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (overflow) atomicOr(&ctl->err, kErrCapacity);
        ctl->n_slots = nbin + nb;
        ctl->next_id += nb;
        ctl->n_births = 0;
        ctl->t += 1;
    }
}

// per-species counts of live agents (LDS histogram, one atomic per species
// per workgroup)
__global__ void __launch_bounds__(kBlock) k_counts(Dev d, int cur)
{
    __shared__ uint32_t h[kMaxSpecies];
    if (threadIdx.x < kMaxSpecies) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = d.ctl->n_slots;
    const uint8_t* sp = d.a[cur].sp;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint32_t s = sp[i];
        if (s < uint32_t(kMaxSpecies)) atomicAdd(&h[s], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxSpecies && h[threadIdx.x])
        atomicAdd(&d.counts[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_zero_counts(Dev d)
{
    if (threadIdx.x < kMaxSpecies) d.counts[threadIdx.x] = 0ull;
}

}  // namespace

// ---------------------------------------------------------------------------
// launch entry points.  Agent-indexed kernels are sized for the capacity
// and read the live sizes from the control block, so a step needs no host
// synchronisation.
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(uint32_t n) { return (n + kBlock - 1) / kBlock; }

void launch_init(const Dev& d, hipStream_t s)
{
    if (d.n_init) k_init<<<blocks_for(d.n_init), kBlock, 0, s>>>(d);
}
void launch_fill_records(const Dev& d, hipStream_t s)
{
    k_fill_records<<<blocks_for(d.capacity), kBlock, 0, s>>>(d);
}
void launch_move(const Dev& d, int cur, int record, hipStream_t s)
{
    k_move<<<blocks_for(d.capacity), kBlock, 0, s>>>(d, cur, record);
}
void launch_scan_reduce(const Dev& d, hipStream_t s)
{
    k_scan_reduce<<<d.ntiles, kScanThreads, 0, s>>>(d);
}
void launch_scan_top(const Dev& d, hipStream_t s) { k_scan_top<<<1, kScanThreads, 0, s>>>(d); }
void launch_scan_down(const Dev& d, hipStream_t s)
{
    k_scan_down<<<d.ntiles, kScanThreads, 0, s>>>(d);
}
void launch_scatter(const Dev& d, int cur, int record, hipStream_t s)
{
    k_scatter<<<blocks_for(d.capacity), kBlock, 0, s>>>(d, cur, record);
}
void launch_propose(const Dev& d, int nxt, hipStream_t s)
{
    k_propose<<<blocks_for(d.capacity), kBlock, 0, s>>>(d, nxt);
}
void launch_apply(const Dev& d, int nxt, int record, hipStream_t s)
{
    k_apply<<<blocks_for(d.capacity), kBlock, 0, s>>>(d, nxt, record);
}
void launch_births(const Dev& d, int nxt, int record, hipStream_t s)
{
    k_births<<<1, kBirthThreads, 0, s>>>(d, nxt, record);
}
void launch_counts(const Dev& d, int cur, hipStream_t s)
{
    k_zero_counts<<<1, 64, 0, s>>>(d);
    unsigned nb = blocks_for(d.capacity);
    if (nb > 2048) nb = 2048;
    if (nb == 0) nb = 1;
    k_counts<<<nb, kBlock, 0, s>>>(d, cur);
}

}  // namespace mabm
