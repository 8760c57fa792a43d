// kernels.hip -- the per-step kernels of the molecule-agent update for
// gfx950 (wave64).  A binning step (O2..O10 of the step definition) of
// parity p (agents start in buffer p and are sorted into buffer p ^ 1) is
// five launches:
//
//   move     one Philox block per agent gives the event draw and the
//            Brownian step; boundaries, event effects, birth records; the
//            cell key of the moved position and its rank in the cell, by one
//            atomic per run of equal keys in a wave (agents arrive sorted by
//            cell from the previous binning, so runs are long and the
//            atomics spread over many cells), and the per-tile sums of the
//            counts the same way
//   scan     each tile (2,048 cells, or a power of two times that) adds the
//            sums of the tiles before it, scans its counts into cell starts
//            and clears them; extra workgroups sort the step's birth records
//            in runs
//   scatter  agents to cell order in the other buffer (holes and degraded
//            agents dropped: stream compaction); extra workgroups place the
//            step's children, ranked by (simulation, parent id), with fresh
//            ids after the binned agents, and one keeps the books (live
//            agents, capacity, next ids, the next step's scalars)
//   propose  per workgroup, a chunk of 1,024 sorted agents (or a share of
//            one): its claimers are compacted in LDS, 27-cell ones first,
//            then each is searched by a group of 4 lanes (16 for 27 cells),
//            two stencil cells per lane, for the nearest eligible partner;
//            Bernoulli draw; handshake keys into both claim slots.  For
//            sparse claimers or small simulations, the claimers listed by
//            the kernel that flagged them instead, each with 16 to 64 lanes
//            (k_propose_list)
//   finish   over the step's proposals: confirmation and pair products
//
// A step that keeps the previous binning (the library allows it while no
// agent can have moved out of reach of the cell lists it was binned in) is
// move, propose and finish on the agents in place: move also writes the
// claimer flags, marks removed agents as holes (listed for later children
// to refill) and chains the agents its rules place into extra per-cell
// chains; propose's extra workgroups sort the birth runs, finish places the
// step's children (into listed holes first, chained too) and its last
// workgroup keeps the books.
//
// Cells are sorted by the Morton index of their coordinates, so the cells of
// a neighbourhood are close in memory.  An agent is a 16-byte record
// {x, y, z, meta} plus a 4-byte id, so a
// streaming kernel moves whole records with 16-byte accesses and a candidate
// check in the neighbour search is one 16-byte gather.  No kernel spins or
// waits on another workgroup, and no hot loop puts many atomics on one
// address or one 4 KiB page (they serialise at the memory side).  Nothing
// here is a dense contraction.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_math.hpp"
#include "engine.hpp"

namespace mabm {

const char* const kKernelNames[kNumKernels] = {"move", "scan", "scatter", "propose", "finish"};

namespace {

constexpr int kBlock = 256;
constexpr int kPChunk = int(kClaimChunk);  // sorted agents per workgroup of propose
constexpr int kPropBlock = kPChunk / 4;    // threads of a propose workgroup (four agents each)

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// lanes strictly below this one
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8), and each XCD has its own L2.  This renumbering gives every XCD a
// contiguous run of chunks, so chunks that gather from the same neighbouring
// cells share one L2.  It is a bijection of [0, gridDim.x).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t n)
{
    const uint32_t b = blockIdx.x;
    const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Lanes whose key equals the previous lane's form a run; each run head adds
// the run length to counter[key * stride] with one atomic.  Returns the
// counter's old value plus the lane's offset in its run.  A key split over
// several runs gets several disjoint ranges, so any lane order is correct;
// sorted keys make runs long and atomics few.  kNone lanes take no part.
__device__ __forceinline__ uint32_t run_add(uint32_t key, uint32_t* counter, uint32_t stride)
{
    const int lane = lane_id();
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || key != prev;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int head_lane = 63 - __builtin_clzll(heads & upto);
    const uint64_t after = heads & ~upto;
    const int next_head = after ? __builtin_ctzll(after) : 64;
    uint32_t base = 0;
    if (head && key != kNone)
        base = atomicAdd(&counter[size_t(key) * stride], uint32_t(next_head - lane));
    base = __shfl(base, head_lane, 64);
    return base + uint32_t(lane - head_lane);
}

// Appends the lanes with `flag` to a list with one atomic on its length per
// wave; returns each flagged lane's index in the list (others: 0).  Called
// by all lanes of the wave.
__device__ __forceinline__ uint32_t wave_append(uint32_t* length, bool flag)
{
    const uint64_t m = __ballot(flag);
    if (!m) return 0u;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(length, uint32_t(__popcll(m)));
    base = __shfl(base, leader, 64);
    return base + uint32_t(__popcll(m & lanes_below()));
}

// Runs f(u) once for every distinct simulation index u among the active
// lanes, with u wave-uniform and only the lanes of simulation u active, so
// that the simulation's tables are read with scalar loads.  Agents are
// sorted by simulation, so nearly every wave takes one pass.
template <class F>
__device__ __forceinline__ void per_sim(uint32_t sim, F&& f)
{
    for (;;) {
        const uint32_t u = __builtin_amdgcn_readfirstlane(sim);
        if (sim == u) {
            f(u);
            break;
        }
    }
}

__device__ __forceinline__ uint32_t sim_of(uint32_t meta) { return meta >> kMetaSimShift; }

__device__ __forceinline__ uint32_t* tile_acc(const Dev& d, int p)
{
    return d.tile_acc + size_t(p) * d.ntiles * kTileStride;
}

__device__ __forceinline__ uint4 make_rec(float x, float y, float z, uint32_t meta)
{
    return uint4{__float_as_uint(x), __float_as_uint(y), __float_as_uint(z), meta};
}

__device__ __forceinline__ void set_species(const Agents& A, uint32_t j, uint32_t s)
{
    reinterpret_cast<uint8_t*>(A.rec + j)[kMetaSpeciesByte] = uint8_t(s);
}


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
    const Agents A = d.a[0];
    A.rec[T.slot_base + i] = make_rec(x, y, z, uint32_t(s) | (T.sim << kMetaSimShift));
    A.id[T.slot_base + i] = i;
}

__global__ void __launch_bounds__(kBlock) k_fill_records(Dev d)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.slots) return;
    d.rkey[i] = kNone;
    d.revent[i] = kNoEvent;
    d.rpartner[i] = kNone;
    d.nxt[i] = kUnlinked;
}

// empty extra chains in every (padded) cell
__global__ void __launch_bounds__(kBlock) k_fill_heads(Dev d, uint32_t n)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d.head[i] = kEnd;
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

// Adds, for every simulation u among the active lanes, their number to
// counter[u] (one atomic per simulation present).  The lanes are grouped by
// comparing their own simulation indices: the active lanes of a branch may
// belong to several simulations even inside per_sim, whose waterfall the
// compiler may dissolve into per-lane table loads.
__device__ __forceinline__ void add_by_sim(uint32_t* counter, uint32_t sim)
{
    uint64_t left = __ballot(1);
    while (left) {
        const uint32_t u = __shfl(sim, __builtin_ctzll(left), 64);
        const uint64_t mine = __ballot(sim == u);
        if (lane_id() == __builtin_ctzll(mine)) atomicAdd(&counter[u], uint32_t(__popcll(mine)));
        left &= ~mine;
    }
}

// A child of this step (a split's second product or an emission) from the
// lanes that take this branch: its record is appended to the step's birth
// records with one atomic per wave, and its simulation's children counted.
__device__ __forceinline__ void append_child(const Dev& d, int p, uint32_t sim, const Birth& b)
{
    const uint32_t k = wave_append(&d.ctl->n_births[p], true);
    add_by_sim(d.sc.born[p], sim);
    if (k < d.capacity) d.births[k] = b;
}

// A slot that became a hole in a step that keeps the binning, from the
// lanes that take this branch: listed (one atomic per wave) for the
// children of this and later steps to refill.
__device__ __forceinline__ void list_hole(const Dev& d, uint32_t i)
{
    const uint32_t k = wave_append(&d.ctl->h_n, true);
    d.hlist[k % d.slots] = i;
}

// A claimer of this step, from the lanes that take this branch, joins the
// claimer list (single simulations in list mode): region blockIdx mod
// kListRegions, one atomic per wave.  A workgroup of kBlock threads appends
// at most kBlock entries, so a region holds those of at most clist_cap /
// kBlock workgroups.
__device__ __forceinline__ void append_claimer(const Dev& d, uint32_t entry)
{
    const uint32_t r = blockIdx.x & (kListRegions - 1u);
    const uint32_t k = wave_append(&d.ccount[r * kListStride], true);
    d.clist[r * d.clist_cap + k] = entry;
}

// ---------------------------------------------------------------------------
// move: O2 (event draw), O3 (Brownian step), O4 (boundaries), O5 and the
// unimolecular part of O8, then the cell key of the moved position and the
// agent's rank within its cell.
// ---------------------------------------------------------------------------
// One live agent's step up to its cell key (the body of move).  In a step
// that keeps the previous binning (bin = 0, `moved` steps after it) the
// agent stays in slot i, so its claimer flag (2 if its species searches the
// 27-cell stencil this step, as the search decides) and recorded fields are
// written here instead of by scatter.  Returns whether a unimolecular rule
// removed the agent; a child of a split or an emission is appended to the
// step's birth records.
template <bool B>
__device__ __forceinline__ bool move_agent(const Dev& d, const Tables& T, const Agents& A, int p,
                                           int record, int bin, uint32_t moved, uint32_t i,
                                           uint32_t id, uint32_t t, const uint4& r, uint32_t s,
                                           uint32_t& key)
{
    const float x = __uint_as_float(r.x), y = __uint_as_float(r.y), z = __uint_as_float(r.z);
    const int c0 = compartment(T, x, y, z);
    const U4 w = draw(T, id, t, kMove, 0u);

    int ev = -1;
    const SpecHot H = T.hot[s][c0];
    const int nu = H.uni_n;
    if (nu) {
        // the cumulative thresholds in rule order: the first from the
        // digest, any further ones from the full table
        const uint32_t wu = event_bits(w);
        if (H.always || wu < H.thr0) {
            ev = H.rule0;
        } else {
            for (int j = 1; j < nu; ++j)
                if (uint64_t(wu) < T.uni_thr[s][c0][j]) {
                    ev = T.uni_rule[s][c0][j];
                    break;
                }
        }
    }

    float z0, z1, z2;
    normals3(w, z0, z1, z2);
    const float sg = H.sigma;
    float x1 = __builtin_fmaf(sg, z0, x), y1 = __builtin_fmaf(sg, z1, y), w1 = __builtin_fmaf(sg, z2, z);
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

    uint32_t fs = s;
    float fx = x1, fy = y1, fz = w1;
    bool dies = false, placed = false;  // placed: moved by its rule, not only by diffusion
    if (ev >= 0) {
        const RuleDev& R = T.rule[ev];
        float ux, uy, uz;
        switch (R.placement) {
        case kKeep:
            if (R.p0 < 0) dies = true;
            else fs = uint32_t(R.p0);
            break;
        case kTranslocate: {
            placed = true;
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
            placed = true;
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
            append_child(d, p, T.sim, Birth{id, uint32_t(R.p1) | (B ? r.w & kMetaSimMask : 0u), cx, cy, cz});
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
            append_child(d, p, T.sim, Birth{id, uint32_t(R.p1) | (B ? r.w & kMetaSimMask : 0u), cx, cy, cz});
            break;
        }
        }
    }
    const uint32_t sim_bits = B ? r.w & kMetaSimMask : 0u;
    if (dies) {
        // a hole until the next binning drops it, or (in a step that keeps
        // the binning) a later birth takes the slot over
        A.rec[i].w = uint32_t(kDead) | sim_bits | (bin ? 0u : kMetaListed);
        if (!bin) {
            d.sclaim[i] = 0;
            list_hole(d, i);
        }
        add_by_sim(d.sc.dead[p], T.sim);
        return true;
    }
    const uint32_t meta = fs | (ev >= 0 ? kMetaBusy : 0u) | sim_bits;
    if (bin) {
        // O6: the cell of the agent's final position (scatter recomputes it
        // from the record)
        key = cell_of(T, fx, fy, fz);
        if (B) key += T.cell_base;
        A.rec[i] = make_rec(fx, fy, fz, meta);
        if (record) d.event[i] = ev >= 0 ? uint8_t(ev) : kNoEvent;
    } else {
        // the final species' claimer data (a conversion changed it rarely)
        const SpecHot& F = fs == s ? H : T.hot[fs][0];
        const bool claim = ev < 0 && F.claimer;
        const bool wide = T.stencil8 && (F.rmax + float(moved) * F.dmax) * T.inv_h > 0.495f;
        A.rec[i] = make_rec(fx, fy, fz, meta | (claim ? kMetaClaimer : 0u));
        d.sclaim[i] = claim ? (wide ? 2 : 1) : 0;
        if (!B && claim && d.list_mode) append_claimer(d, i | (wide ? kListWide : 0u));
        if (record) {
            d.rkey[i] = linear_cell(T, cell_of(T, fx, fy, fz));
            d.revent[i] = ev >= 0 ? uint8_t(ev) : kNoEvent;
            d.rpartner[i] = kNone;
        }
        if (placed && d.link) {
            // far from its cell list now: it heads the extra chain of its new
            // cell, or, if already chained since the binning, joins the
            // global list (each slot at most once in each)
            uint32_t c = cell_of(T, fx, fy, fz);
            if (B) c += T.cell_base;
            const uint32_t old = d.nxt[i];
            if ((old & ~kGlobBit) == kUnlinked) {
                d.nxt[i] = atomicExch(&d.head[c], i);
            } else if (!(old & kGlobBit)) {
                d.nxt[i] = old | kGlobBit;
                d.glob[atomicAdd(&d.ctl->n_glob, 1u)] = i;
            }
        }
    }
    return false;
}

template <bool B>
__global__ void __launch_bounds__(kBlock) k_move(Dev d, int p, int record, int bin, uint32_t moved)
{
    const uint32_t n = d.ctl->s[p].n_slots;
    const uint32_t t = d.ctl->s[p].t;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const Agents A = d.a[p];
    // claim slots start every step at all-ones: the previous step wrote only
    // those of its proposers and their targets, which are reset here
    if (i < d.ctl->n_prop[p ^ 1]) {
        const uint4 e = d.plist[i];
        d.slot[e.x] = ~0ull;
        d.slot[e.y] = ~0ull;
    }
    uint32_t key = kNone;
    uint4 r = {0u, 0u, 0u, kDead};
    uint32_t id = 0;
    if (i < n) {
        r = A.rec[i];
        id = A.id[i];
    }
    const uint32_t s = r.w & 0xFFu;
    if (s != kDead) {
        if (B)
            per_sim(sim_of(r.w), [&](uint32_t u) {
                move_agent<true>(d, d.tab[u], A, p, record, bin, moved, i, id, t, r, s, key);
            });
        else
            move_agent<false>(d, *d.tab, A, p, record, bin, moved, i, id, t, r, s, key);
    } else if (!bin && i < n) {
        d.sclaim[i] = 0;  // a hole kept in its slot
        // an agent removed by an earlier step's pair rule joins the hole list
        // once (its record is marked listed)
        if (!(r.w & kMetaListed)) {
            A.rec[i].w = r.w | kMetaListed;
            list_hole(d, i);
        }
    }
    if (!bin) return;
    // rank within the cell, and the per-tile sums the scan starts from
    const uint32_t rank = run_add(key, d.cell_count, 1u);
    run_add(key == kNone ? kNone : key >> (kScanTileLog + d.tile_shift), tile_acc(d, p), kTileStride);
    if (i < n) d.rank[i] = key == kNone ? kNone : rank;
}

// ---------------------------------------------------------------------------
// births (O9).  The children of a step take ids in parent-id order, per
// simulation: child of rank r among its simulation's children gets id
// next_id + r.  The rank is found without a global sort: the step's birth
// records (appended by move in any order) are cut into runs of kBirthRun;
// each run is sorted in LDS by its key (simulation << 32 | parent id; keys
// are unique, a parent having at most one child per step), which gives
// every record its rank in its own run and the number of records of
// smaller simulations there; a record's rank among all births is then its
// rank in its run plus, for every other run, the number of keys below its
// own (a binary search).  Slots follow the same order: a binning step
// appends the children after the binned agents; a step that keeps the
// binning first refills the holes listed since the binning, then appends.
// ---------------------------------------------------------------------------
static_assert(kBirthRun == kBlock && kBirthRun <= kPropBlock,
              "one birth record per thread of a sorting workgroup");

__device__ __forceinline__ unsigned long long birth_key(const Birth& b)
{
    return ((unsigned long long)(b.sp >> kMetaSimShift) << 32) | b.parent;
}

// Workgroup w of n_w sorts runs w, w + n_w, ...: bitonic sort of the run's
// (key, index) pairs in LDS, padded with all-ones keys; the sorted keys go
// to bkey, and each record's rank in the run and the number of the run's
// records of smaller simulations to brank.
__device__ void sort_birth_runs(const Dev& d, int p, uint32_t w, uint32_t n_w)
{
    __shared__ unsigned long long key[kBirthRun];
    __shared__ uint32_t pos[kBirthRun];
    const uint32_t nb = min(d.ctl->n_births[p], d.capacity);
    if (nb <= kBirthRun) return;  // a single run is ranked where it is placed
    const uint32_t j = threadIdx.x;
    const bool act = j < kBirthRun;  // a wider workgroup's other threads only synchronise
    for (uint32_t run = w; run * kBirthRun < nb; run += n_w) {
        const uint32_t lo = run * kBirthRun;
        const uint32_t m = min(kBirthRun, nb - lo);
        if (act) {
            key[j] = j < m ? birth_key(d.births[lo + j]) : ~0ull;
            pos[j] = j;
        }
        __syncthreads();
        for (uint32_t k = 2; k <= kBirthRun; k <<= 1) {
            for (uint32_t h = k >> 1; h > 0; h >>= 1) {
                const uint32_t l = j ^ h;
                if (act && l > j) {
                    const bool up = (j & k) == 0;
                    const unsigned long long a = key[j], c = key[l];
                    if ((a > c) == up) {
                        key[j] = c;
                        key[l] = a;
                        const uint32_t t = pos[j];
                        pos[j] = pos[l];
                        pos[l] = t;
                    }
                }
                __syncthreads();
            }
        }
        if (act && j < m) {
            const unsigned long long kj = key[j];
            d.bkey[lo + j] = kj;
            // first position of this record's simulation in the sorted run
            const unsigned long long first = kj & 0xFFFFFFFF00000000ull;
            uint32_t x = 0, y = j;
            while (x < y) {
                const uint32_t mid = (x + y) >> 1;
                if (key[mid] < first) x = mid + 1;
                else y = mid;
            }
            d.brank[lo + pos[j]] = uint2{j, x};
        }
        __syncthreads();  // the run's LDS is reused by the next one
    }
}

// keys of a sorted run below `key`
__device__ __forceinline__ uint32_t count_below(const unsigned long long* run, uint32_t len,
                                                unsigned long long key)
{
    uint32_t x = 0, y = len;
    while (x < y) {
        const uint32_t mid = (x + y) >> 1;
        if (run[mid] < key) x = mid + 1;
        else y = mid;
    }
    return x;
}

// Slots of a step's children: a binning step appends them after the binned
// agents (base = the binned count); a step that keeps the binning first
// refills the listed holes not yet refilled (m of them), then appends after
// its slots (base = the slot count).
struct BirthSlots {
    uint32_t base, m, h_used;
};

__device__ __forceinline__ BirthSlots birth_slots(const Dev& d, const StepState& cur, bool bin,
                                                  uint32_t nb)
{
    if (bin) return BirthSlots{d.ctl->n_binned, 0u, 0u};
    const uint32_t avail = d.ctl->h_n - cur.h_used;
    return BirthSlots{cur.n_slots, nb < avail ? nb : avail, cur.h_used};
}

// Writes birth record bb as the child of rank r among the step's children
// (`smaller` of them belong to simulations of lower index): its slot and
// id follow from the rank.  The child takes no part in its birth step's
// search (busy flag); while a binning is kept it heads the extra chain of
// its cell, or, in a refilled hole that already lies in a chain, joins the
// global list.
template <bool B>
__device__ void put_birth(const Dev& d, int p, const Agents& A, const Birth& bb, uint32_t r,
                          uint32_t smaller, const BirthSlots& bs, int record)
{
    const uint32_t sim = B ? bb.sp >> kMetaSimShift : 0u;
    const uint32_t j = r < bs.m ? d.hlist[(bs.h_used + r) % d.slots] : bs.base + (r - bs.m);
    if (j >= d.slots) return;  // the bookkeeping reports the overflow
    A.rec[j] = make_rec(bb.x, bb.y, bb.z, bb.sp | kMetaBusy);
    A.id[j] = d.sc.next_id[p][sim] + (r - (B ? smaller : 0u));
    if (record) {
        d.rkey[j] = kNone;
        d.revent[j] = kNoEvent;
        d.rpartner[j] = kNone;
    }
    if (d.link) {
        const Tables& T = d.tab[sim];
        uint32_t cell = cell_of(T, bb.x, bb.y, bb.z);
        if (B) cell += T.cell_base;
        if (r >= bs.m) {
            d.nxt[j] = atomicExch(&d.head[cell], j);  // a fresh slot
        } else {
            const uint32_t old = d.nxt[j];
            if ((old & ~kGlobBit) == kUnlinked) {
                d.nxt[j] = atomicExch(&d.head[cell], j);
            } else if (!(old & kGlobBit)) {
                d.nxt[j] = old | kGlobBit;
                d.glob[atomicAdd(&d.ctl->n_glob, 1u)] = j;
            }
        }
    }
}

// Places birth record k of a step with more than one run of children
// (their runs sorted): its rank is its rank in its run plus its lower bound
// in every other run.
template <bool B>
__device__ void place_birth(const Dev& d, int p, const Agents& A, uint32_t k, uint32_t nb,
                            const BirthSlots& bs, int record)
{
    const Birth bb = d.births[k];
    const unsigned long long key = birth_key(bb);
    const uint2 br = d.brank[k];
    uint32_t r = br.x, smaller = br.y;
    const uint32_t runs = (nb + kBirthRun - 1) >> kBirthRunLog;
    const uint32_t own = k >> kBirthRunLog;
    for (uint32_t q = 0; q < runs; ++q) {
        if (q == own) continue;
        const unsigned long long* run = d.bkey + (size_t(q) << kBirthRunLog);
        const uint32_t len = min(kBirthRun, nb - (q << kBirthRunLog));
        r += count_below(run, len, key);
        if (B) smaller += count_below(run, len, key & 0xFFFFFFFF00000000ull);
    }
    put_birth<B>(d, p, A, bb, r, smaller, bs, record);
}

// Places the children of a step with at most one run of them, all by one
// workgroup: their keys in LDS, each child's rank by counting the keys below
// its own.
template <bool B>
__device__ void place_births_small(const Dev& d, int p, const Agents& A, uint32_t nb,
                                   const BirthSlots& bs, int record)
{
    __shared__ unsigned long long skey[kBirthRun];
    const uint32_t j = threadIdx.x;
    Birth bb{};
    if (j < nb) {
        bb = d.births[j];
        skey[j] = birth_key(bb);
    }
    __syncthreads();
    if (j < nb) {
        const unsigned long long key = skey[j], first = key & 0xFFFFFFFF00000000ull;
        uint32_t r = 0, smaller = 0;
        for (uint32_t q = 0; q < nb; ++q) {
            const unsigned long long o = skey[q];
            r += o < key ? 1u : 0u;
            smaller += o < first ? 1u : 0u;
        }
        put_birth<B>(d, p, A, bb, r, smaller, bs, record);
    }
}

// All of a step's children, placed by workgroup w of n_w: one run of
// children by the workgroup `small_w`, more by all of them.
template <bool B>
__device__ void place_births(const Dev& d, int p, const Agents& A, uint32_t nb,
                             const BirthSlots& bs, int record, uint32_t w, uint32_t n_w,
                             uint32_t small_w)
{
    if (nb <= kBirthRun) {
        if (w == small_w && nb) place_births_small<B>(d, p, A, nb, bs, record);
        return;
    }
    for (uint32_t k = w * kBlock + threadIdx.x; k < nb; k += n_w * kBlock)
        place_birth<B>(d, p, A, k, nb, bs, record);
}

// The step's bookkeeping (O9, O10), run by one whole workgroup while the
// other workgroups of its kernel place the step's children:
//   - per simulation, the live agents at this step's start (those at the
//     previous step's start, less its removals, plus its children) are
//     checked against the simulation's capacity (a step whose end exceeds
//     it raises the sticky capacity error here, or at the next query if it
//     is the last step run) and summed into the agent-update count; the
//     next step's first id is this one's plus this step's children;
//   - the next step's slot count: a binning step's binned agents plus its
//     children; a kept step's slots plus the children that did not refill
//     a hole (the arrays hold `slots` entries: more is the slot error).
template <bool B>
__device__ void bookkeeping(const Dev& d, int p, bool bin)
{
    __shared__ unsigned long long live_part[kBlock / 64];
    __shared__ uint32_t over_part[kBlock / 64];
    Ctl* ctl = d.ctl;
    const StepState cur = ctl->s[p];
    const SimCounters& sc = d.sc;
    unsigned long long live_sum = 0;
    uint32_t over = 0;
    for (uint32_t k = threadIdx.x; k < d.n_sims; k += kBlock) {
        const uint32_t live = sc.live[k] - sc.dead[p ^ 1][k] + sc.born[p ^ 1][k];
        sc.live[k] = live;
        sc.dead[p ^ 1][k] = 0u;
        sc.born[p ^ 1][k] = 0u;
        sc.next_id[p ^ 1][k] = sc.next_id[p][k] + sc.born[p][k];
        over |= live > d.tab[k].capacity ? 1u : 0u;
        live_sum += live;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        live_sum += __shfl_xor(live_sum, o, 64);
        over |= __shfl_xor(over, o, 64);
    }
    if (lane_id() == 0) {
        live_part[threadIdx.x >> 6] = live_sum;
        over_part[threadIdx.x >> 6] = over;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        uint32_t bad = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            tot += live_part[w];
            bad |= over_part[w];
        }
        const uint32_t nb_all = ctl->n_births[p];
        const uint32_t nb = min(nb_all, d.capacity);
        const BirthSlots bs = birth_slots(d, cur, bin, nb);
        uint64_t slots_next = uint64_t(bs.base) + (nb - bs.m);
        uint32_t err = bad ? kErrCapacity : 0u;
        if (nb_all > d.capacity || slots_next > d.slots) {
            err |= kErrSlots;
            if (slots_next > d.slots) slots_next = d.slots;
        }
        if (err) atomicOr(&ctl->err, err);
        ctl->agent_updates += tot;
        ctl->n_births[p ^ 1] = 0u;
        ctl->n_prop[p ^ 1] = 0u;
        if (bin) {
            // a new binning: no holes yet (the binned agents are compacted),
            // no extra chains, no agents placed twice
            ctl->h_n = 0u;
            ctl->n_glob = 0u;
        }
        ctl->s[p ^ 1] = StepState{cur.t + 1u, uint32_t(slots_next), cur.next_id + nb,
                                  bin ? 0u : bs.h_used + bs.m};
    }
}

// Births and bookkeeping of a binning step, run by the extra workgroups of
// the scatter launch: the last one does the bookkeeping, all of them place
// the step's children after the binned agents in the sorted buffer.
template <bool B>
__device__ void scatter_births(const Dev& d, int p, int record, uint32_t w, uint32_t n_w)
{
    const uint32_t nb = min(d.ctl->n_births[p], d.capacity);
    const BirthSlots bs = birth_slots(d, d.ctl->s[p], true, nb);
    place_births<B>(d, p, d.a[p ^ 1], nb, bs, record, w, n_w, 0u);
    if (w == n_w - 1) {
        // the scan has read this parity's tile sums (and cleared the
        // other's): clear them too, so that steps keeping this binning need
        // not
        uint32_t* acc = tile_acc(d, p);
        for (uint32_t k = threadIdx.x; k < d.ntiles; k += kBlock) acc[size_t(k) * kTileStride] = 0u;
        bookkeeping<B>(d, p, true);
    }
}

// ---------------------------------------------------------------------------
// scatter: binned agents to cell order in the other buffer; the claimer flag
// (non-busy agent of a claiming species) is set in the record and in the
// one-byte array the propose chunks scan.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// scan of the cell counts, one launch, no waiting between workgroups: each
// tile sums the earlier tiles' totals (accumulated by move), scans its 2048
// counts into cell starts, clears them, and clears its accumulator of the
// other parity for the next step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan over the 256-thread block; the block total in *total
// Exclusive prefix of v and the block totals of v and r, with one exchange
// through LDS.
__device__ __forceinline__ uint32_t block_excl_scan_sum(uint32_t v, uint32_t r, uint32_t* total_v,
                                                        uint32_t* total_r)
{
    __shared__ uint32_t wsum[2][kScanThreads / 64];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    const uint32_t rr = wave_incl_scan(r);
    if (lane == 63) {
        wsum[0][wv] = inc;
        wsum[1][wv] = rr;
    }
    __syncthreads();
    uint32_t off = 0, tot = 0, totr = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < wv) off += wsum[0][k];
        tot += wsum[0][k];
        totr += wsum[1][k];
    }
    *total_v = tot;
    *total_r = totr;
    __syncthreads();  // wsum may be rewritten by the next call
    return off + inc - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan(Dev d, int p)
{
    if (blockIdx.x >= d.ntiles) {
        // the workgroups after the tiles sort the step's birth runs
        sort_birth_runs(d, p, blockIdx.x - d.ntiles, gridDim.x - d.ntiles);
        return;
    }
    const uint32_t tile = blockIdx.x;
    const uint32_t npass = 1u << d.tile_shift;
    constexpr int kVec = kScanItems / 4;
    uint4* cnt4 = reinterpret_cast<uint4*>(d.cell_count + (size_t(tile) << (kScanTileLog + d.tile_shift)) +
                                           threadIdx.x * kScanItems);
    uint4* st4 = reinterpret_cast<uint4*>(d.cell_start + (size_t(tile) << (kScanTileLog + d.tile_shift)) +
                                          threadIdx.x * kScanItems);
    // the extra chains of the previous binning end with this one
    uint4* hd4 = reinterpret_cast<uint4*>(d.head + (size_t(tile) << (kScanTileLog + d.tile_shift)) +
                                          threadIdx.x * kScanItems);
    constexpr uint32_t kPassVec = kScanTile / 4;  // uint4 per pass
    // the first pass's counts are requested before the preceding tiles'
    // sums, so both loads are in flight together
    uint4 v[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) v[k] = cnt4[k];
    const uint32_t* acc = tile_acc(d, p);
    uint32_t before = 0;
    for (uint32_t k = threadIdx.x; k < tile; k += kScanThreads) before += acc[size_t(k) * kTileStride];
    uint32_t base = 0;  // cells before this pass
    for (uint32_t pass = 0; pass < npass; ++pass) {
        // the next pass's counts are requested before this pass is scanned
        uint4 nx[kVec];
        if (pass + 1 < npass) {
#pragma unroll
            for (int k = 0; k < kVec; ++k) nx[k] = cnt4[(pass + 1) * kPassVec + k];
        }
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kVec; ++k) sum += v[k].x + v[k].y + v[k].z + v[k].w;
        uint32_t total, prefix;
        uint32_t run = block_excl_scan_sum(sum, pass == 0 ? before : 0u, &total, &prefix);
        if (pass == 0) base = prefix;
        run += base;
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            uint4 o;
            o.x = run;
            run += v[k].x;
            o.y = run;
            run += v[k].y;
            o.z = run;
            run += v[k].z;
            o.w = run;
            run += v[k].w;
            st4[pass * kPassVec + k] = o;
            cnt4[pass * kPassVec + k] = uint4{0u, 0u, 0u, 0u};
            if (d.link) hd4[pass * kPassVec + k] = uint4{kEnd, kEnd, kEnd, kEnd};
        }
        base += total;
        if (pass + 1 < npass) {
#pragma unroll
            for (int k = 0; k < kVec; ++k) v[k] = nx[k];
        }
    }
    if (threadIdx.x == 0) {
        tile_acc(d, p ^ 1)[size_t(tile) * kTileStride] = 0u;
        if (tile == d.ntiles - 1) {
            d.cell_start[size_t(d.ntiles) << (kScanTileLog + d.tile_shift)] = base;
            d.ctl->n_binned = base;
        }
    }
}

template <bool B>
__device__ __forceinline__ void scatter_slot(const Dev& d, int p, int record, uint32_t i)
{
    const uint32_t rank = d.rank[i];
    if (rank == kNone) return;
    const Tables& T = *d.tab;
    const Agents A = d.a[p];
    const Agents O = d.a[p ^ 1];
    uint4 r = A.rec[i];
    // the cell key move binned the agent under, from its recorded position
    uint32_t key;
    if (B) {
        const Tables& Ts = d.tab[sim_of(r.w)];
        key = Ts.cell_base + cell_of(Ts, __uint_as_float(r.x), __uint_as_float(r.y),
                                     __uint_as_float(r.z));
    } else {
        key = cell_of(T, __uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z));
    }
    const uint32_t j = d.cell_start[key] + rank;
    const bool claim = !(r.w & kMetaBusy) && T.claimer[r.w & 0xFFu];
    if (claim) r.w |= kMetaClaimer;
    O.rec[j] = r;
    O.id[j] = A.id[i];
    d.sclaim[j] = claim ? 1 : 0;
    if (!B && claim && d.list_mode) append_claimer(d, j);
    if (d.link) d.nxt[j] = kUnlinked;  // binned: in no extra chain
    if (record) {
        if (B) {
            const Tables& Ts = d.tab[sim_of(r.w)];
            d.rkey[j] = linear_cell(Ts, key - Ts.cell_base);
        } else {
            d.rkey[j] = linear_cell(T, key);
        }
        d.revent[j] = d.event[i];
        d.rpartner[j] = kNone;
    }
}

// The first agent_blocks workgroups cover the slots (one agent per
// thread); the rest place the step's children and do its bookkeeping.
template <bool B>
__global__ void __launch_bounds__(kBlock) k_scatter(Dev d, int p, int record, uint32_t agent_blocks)
{
    if (blockIdx.x >= agent_blocks) {
        scatter_births<B>(d, p, record, blockIdx.x - agent_blocks, gridDim.x - agent_blocks);
        return;
    }
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < d.ctl->s[p].n_slots) scatter_slot<B>(d, p, record, i);
}

// Compact, in LDS, the claimers of this workgroup's chunk [first, last) of
// kPChunk = kClaimPer x kPropBlock sorted agents: each thread reads the claimer
// flags of its kClaimPer agents as one word (1: a claimer, 2: a claimer that
// searches the 27-cell stencil this step), a wave-level prefix of both
// counts places them within the wave, and the waves' totals, exchanged
// through LDS, place the waves; the wide claimers come first, each kind in
// agent order.  The order is the same in every workgroup that compacts the
// chunk, which lets several share its claimers.  `word` is loaded by the
// caller before anything else so that its latency overlaps the kernel's
// other set-up loads.  Returns the list length, and the wide claimers'
// count in *n_wide.
constexpr int kClaimPer = kPChunk / kPropBlock;
constexpr uint32_t kPropLds = 256;  // proposals a workgroup stages in LDS
static_assert(kClaimPer == 2 || kClaimPer == 4, "two or four claimer flags per thread");
using FlagWord = std::conditional_t<kClaimPer == 4, uint32_t, uint16_t>;

__device__ __forceinline__ uint32_t compact_claimers(uint32_t word, uint32_t first, uint32_t last,
                                                     uint32_t* list, uint32_t* count,
                                                     uint32_t* n_wide)
{
    const uint32_t k0 = first + uint32_t(kClaimPer) * threadIdx.x;
    uint32_t flags = 0;
    if (k0 < last) {
        // flags past `last` are dropped
        flags = word;
        const uint32_t valid = last - k0;
        if (valid < uint32_t(kClaimPer)) flags &= (1u << (8u * valid)) - 1u;
    }
    // counts packed as (wide << 16) | narrow (each at most kPChunk)
    uint32_t mine = 0;
#pragma unroll
    for (int b = 0; b < kClaimPer; ++b) {
        const uint32_t v = (flags >> (8 * b)) & 0xFFu;
        mine += v == 2u ? 0x10000u : (v ? 1u : 0u);
    }
    uint32_t incl = mine;
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    __shared__ uint32_t wsum[kPropBlock / 64];
    const int wv = int(threadIdx.x) >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t base = incl - mine, total = 0;
#pragma unroll
    for (int k = 0; k < kPropBlock / 64; ++k) {
        if (k < wv) base += wsum[k];
        total += wsum[k];
    }
    const uint32_t tw = total >> 16, tn = total & 0xFFFFu;
    uint32_t bw = base >> 16, bn = tw + (base & 0xFFFFu);
#pragma unroll
    for (int b = 0; b < kClaimPer; ++b) {
        const uint32_t v = (flags >> (8 * b)) & 0xFFu;
        if (v == 2u) list[bw++] = k0 + uint32_t(b);
        else if (v) list[bn++] = k0 + uint32_t(b);
    }
    if (threadIdx.x == 0) {
        *count = tw + tn;
        *n_wide = tw;
    }
    __syncthreads();
    return tw + tn;
}

// ---------------------------------------------------------------------------
// propose (O7): for each claimer, the eligible partner minimising (d^2, id)
// over its 8-cell or 27-cell stencil, then a Bernoulli draw,
// then the handshake key into both claim slots by atomic minimum.  A
// workgroup takes 1,024 sorted agents; their claimers are searched by
// subgroups of 4 (or 16) lanes, two stencil cells per lane, and the lanes'
// best candidates are reduced by shuffles, so each claimer's dependent
// chain of loads is a few round trips long.
// ---------------------------------------------------------------------------
// rule: the pair rule's index, plus kBestClaimer when the candidate is a
// claimer itself this step (finish's mutual-pair test needs it)
constexpr int kBestClaimer = 0x100;
struct Best {
    uint32_t idx, id;
    float d2;
    int rule;
};

// The pair-rule table and the contact radii live in LDS while a workgroup
// searches: rule index of (claimer species, target species), -1 for none.
struct PairLds {
    uint8_t rule_of[kMaxSpecies * kMaxSpecies];
    float r2[kMaxRules];
    float r2max[kMaxSpecies];  // per claimer species, its largest r2
    float rmax[kMaxSpecies];   // and its largest contact radius
    float dmax[kMaxSpecies];   // and how far one step moves its targets at most
};

template <bool B>
__device__ __forceinline__ void consider(const Tables& T, const PairLds& P, const Agents& A,
                                         const uint4& rk, uint32_t k, uint32_t self, uint32_t s,
                                         float x, float y, float z, int comp, float r2max,
                                         Best& b)
{
    const float bx = __uint_as_float(rk.x), by = __uint_as_float(rk.y), bz = __uint_as_float(rk.z);
    float dx = bx - x, dy = by - y, dz = bz - z;
    if (T.geometry == kBox) {
        if (dx > T.halfL) dx -= T.L; else if (dx < -T.halfL) dx += T.L;
        if (dy > T.halfL) dy -= T.L; else if (dy < -T.halfL) dy += T.L;
        if (dz > T.halfL) dz -= T.L; else if (dz < -T.halfL) dz += T.L;
    }
    const float d2 = dx * dx + dy * dy + dz * dz;
    // no rule of the claimer's species reaches beyond r2max, so nearly
    // every candidate stops here, before the rule lookup
    if (!(d2 <= r2max)) return;
    const uint32_t sb = rk.w & 0xFFu;
    const uint32_t rv = sb < uint32_t(kMaxSpecies) ? P.rule_of[s * kMaxSpecies + sb] : kNoRule;
    const int r = rv == kNoRule ? -1 : int(rv);
    if (k == self || r < 0 || (rk.w & kMetaBusy)) return;
    // in a batch a slot of this simulation's cell lists may hold another
    // simulation's child (a refilled hole), and the global list holds every
    // simulation's agents
    if (B && sim_of(rk.w) != T.sim) return;
    if (T.geometry == kNested && compartment(T, bx, by, bz) != comp) return;
    if (!(d2 <= P.r2[r])) return;
    if (b.idx != kNone && d2 > b.d2) return;
    const uint32_t bid = A.id[k];
    if (b.idx == kNone || d2 < b.d2 || bid < b.id) {
        b.idx = k;
        b.id = bid;
        b.d2 = d2;
        b.rule = r | ((rk.w & kMetaClaimer) ? kBestClaimer : 0);
    }
}

// Lexicographic minimum of (d^2, id) over the lanes of each aligned group
// of w lanes (xor butterfly; w differs between groups of one wave, so the
// exchange runs over the widest group's steps, `top`, and a lane combines
// only steps within its own group).
__device__ __forceinline__ void reduce_best(Best& b, int w, int top)
{
    for (int o = top >> 1; o >= 1; o >>= 1) {
        Best c;
        c.idx = __shfl_xor(b.idx, o, 64);
        c.id = __shfl_xor(b.id, o, 64);
        c.d2 = __shfl_xor(b.d2, o, 64);
        c.rule = __shfl_xor(b.rule, o, 64);
        if (o < w && c.idx != kNone &&
            (b.idx == kNone || c.d2 < b.d2 || (c.d2 == b.d2 && c.id < b.id)))
            b = c;
    }
}

// O7 search for one claimer j (record rj, id ida) by its group of `width`
// lanes (lane li scans stencil cells li and li + width; `top` is the widest
// group of the workgroup), then lane 0's Bernoulli draw and handshake keys.
// `moved`: steps since the agents were binned.  `wide`: the claimer
// searches the 27-cell stencil (always where the grid does not allow the
// 8-cell one; in a step that keeps a binning, also when its species'
// contact radius plus its targets' moves since the binning exceed the
// 8-cell stencil's reach of half a cell, less 1 %, as move decided when it
// flagged the claimer).  Groups are at least half as wide as the stencil.
// Sl (the claimer list's search, groups of 16 to 64 lanes): a group at
// least as wide as the stencil rounded up to a power of two (8, or 32 for
// 27 cells) gives each cell width / 8 (or width / 32) lanes, which take
// every (width / 8)-th (or (width / 32)-th) of its candidates, so a crowded
// cell is scanned by several lanes; narrower groups keep two cells per lane.
template <bool B, bool Sl = false>
__device__ __forceinline__ void search_claimer(const Dev& d, const Tables& T, const PairLds& P,
                                               const Agents& A, uint32_t t, uint32_t j,
                                               const uint4& rj, uint32_t ida, int li, int width,
                                               int top, bool wide, uint32_t moved, uint32_t n_glob,
                                               uint4* plocal, uint32_t* nprop, uint32_t* n_prop)
{
    const int G = int(T.G);
    const bool periodic = T.geometry == kBox;
    const uint32_t s = rj.w & 0xFFu;
    wide = wide || !T.stencil8;
    const int ncell = wide ? 27 : 8;
    const float stale = float(moved) * P.dmax[s];
    const float r2max = P.r2max[s];
    const float x = __uint_as_float(rj.x), y = __uint_as_float(rj.y), z = __uint_as_float(rj.z);
    const int comp = compartment(T, x, y, z);
    const float pp[3] = {x, y, z};
    int c[3];
    float f[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = int(cell_coord(T, pp[a]));
        f[a] = (pp[a] - T.lo) * T.inv_h - float(c[a]);
    }
    // Stencil cells that cannot hold a partner are not read.  Per axis, the
    // gap from the claimer to the cell (in cells; 0 along an axis where the
    // cell is level with the claimer's own), less how far a candidate may
    // have moved since it was binned, gives a lower bound on the distance to
    // any candidate listed in the cell; the cell is skipped when that bound
    // exceeds the claimer's largest contact radius, padded by 0.1 % and
    // 1e-3 cells (far above the rounding of the cell coordinates).
    const float shrink = stale * T.inv_h;
    const float rho = P.rmax[s] * T.inv_h * 1.001f + 1e-3f;
    const float rho2 = rho * rho;
    // candidate range of stencil cell m and the head of its extra chain
    // (empty outside the grid or out of reach)
    auto range = [&](int m, uint32_t& lo, uint32_t& hi, uint32_t& hd) {
        lo = hi = 0;
        hd = kEnd;
        if (m >= ncell) return;
        int cc[3];
        float gap2 = 0.0f;
        for (int a = 0; a < 3; ++a) {
            int o;
            if (!wide) {
                // the neighbour on the side of the cell the point is nearer
                o = ((m >> a) & 1) * (f[a] < 0.5f ? -1 : 1);
            } else {
                o = (a == 0 ? m % 3 : (a == 1 ? (m / 3) % 3 : m / 9)) - 1;
            }
            float g = o < 0 ? f[a] : (o > 0 ? 1.0f - f[a] : 0.0f);
            g = fmaxf(g - shrink, 0.0f);
            gap2 += g * g;
            int v = c[a] + o;
            if (periodic) v = (v + G) % G;
            else if (v < 0 || v >= G) return;
            cc[a] = v;
        }
        if (gap2 > rho2) return;
        uint32_t cell = cell_key(uint32_t(cc[0]), uint32_t(cc[1]), uint32_t(cc[2]));
        if (B) cell += T.cell_base;
        lo = d.cell_start[cell];
        hi = d.cell_start[cell + 1];
        if (d.link) hd = d.head[cell];
    };
    uint32_t k0, e0, k1, e1, h0, h1;
    // lane li's cells m0 and m1 (m1 none for a sliced lane), its first
    // candidate's offset in them and the stride between its candidates
    int m0 = li, m1 = li + width;
    uint32_t slice = 0, stride = 1;
    if (Sl) {
        const int npad = wide ? 32 : 8;
        if (width >= npad) {
            m0 = li & (npad - 1);
            m1 = 1 << 30;
            slice = uint32_t(li / npad);
            stride = uint32_t(width / npad);
        }
    }
    range(m0, k0, e0, h0);
    range(m1, k1, e1, h1);
    k0 += slice;
    k1 += slice;
    if (Sl && slice) h0 = h1 = kEnd;  // a cell's first lane walks its extra chain
    Best b{kNone, 0u, 0.0f, -1};
    // up to two candidates of each cell per round, all four records
    // requested together
    while (k0 < e0 || k1 < e1) {
        const bool a0 = k0 < e0, a1 = k0 + stride < e0, b0 = k1 < e1, b1 = k1 + stride < e1;
        uint4 r0{}, r1{}, r2{}, r3{};
        if (a0) r0 = A.rec[k0];
        if (a1) r1 = A.rec[k0 + stride];
        if (b0) r2 = A.rec[k1];
        if (b1) r3 = A.rec[k1 + stride];
        if (a0) consider<B>(T, P, A, r0, k0, j, s, x, y, z, comp, r2max, b);
        if (a1) consider<B>(T, P, A, r1, k0 + stride, j, s, x, y, z, comp, r2max, b);
        if (b0) consider<B>(T, P, A, r2, k1, j, s, x, y, z, comp, r2max, b);
        if (b1) consider<B>(T, P, A, r3, k1 + stride, j, s, x, y, z, comp, r2max, b);
        k0 += 2 * stride;
        k1 += 2 * stride;
    }
    if (d.link) {
        // agents placed since the binning: the cells' extra chains, and the
        // global list (agents placed twice), shared among the group's lanes
        for (uint32_t k = h0; k != kEnd; k = d.nxt[k] & ~kGlobBit)
            consider<B>(T, P, A, A.rec[k], k, j, s, x, y, z, comp, r2max, b);
        for (uint32_t k = h1; k != kEnd; k = d.nxt[k] & ~kGlobBit)
            consider<B>(T, P, A, A.rec[k], k, j, s, x, y, z, comp, r2max, b);
        for (uint32_t q = uint32_t(li); q < n_glob; q += uint32_t(width)) {
            const uint32_t k = d.glob[q];
            consider<B>(T, P, A, A.rec[k], k, j, s, x, y, z, comp, r2max, b);
        }
    }
    reduce_best(b, width, top);
    if (li == 0) {
        uint32_t out = kNone;
        if (b.idx != kNone) {
            const uint32_t w = draw(T, ida, t, kPair, 0u).w0;
            if (uint64_t(w) < T.rule[b.rule & 0xFF].thr) {
                const uint32_t lo_id = ida < b.id ? ida : b.id, hi_id = ida < b.id ? b.id : ida;
                const unsigned long long pr =
                    (unsigned long long)draw(T, lo_id, t, kPrio, hi_id).w0 << 32;
                atomicMin(&d.slot[j], pr | b.id);
                atomicMin(&d.slot[b.idx], pr | ida);
                out = b.idx;
                // the proposal, staged in LDS for the workgroup's one
                // reservation in the step's list (the rare overflow
                // reserves its own entry)
                // {claimer, target, claimer id, rule | target claims <<
                // 8 | simulation << 16}: what finish needs besides the
                // slots and the target's id
                const uint4 e{j, b.idx, ida, uint32_t(b.rule & 0x1FF) | (T.sim << 16)};
                const uint32_t k = atomicAdd(nprop, 1u);
                if (k < kPropLds) plocal[k] = e;
                else d.plist[atomicAdd(n_prop, 1u)] = e;
            }
        }
        d.prop[j] = out;
    }
}

template <bool B>
__global__ void __launch_bounds__(kPropBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_propose(Dev d, int p, uint32_t split, int bin, uint32_t moved, uint32_t search_blocks,
          uint32_t core_blocks)
{
    __shared__ uint32_t list[kPChunk];
    __shared__ uint4 plocal[kPropLds];
    __shared__ PairLds P;
    __shared__ uint32_t count, nprop, pbase;
    if (blockIdx.x >= search_blocks) {
        // a step that keeps the binning sorts its birth runs here (after
        // move has appended them, before finish places them)
        sort_birth_runs(d, p, blockIdx.x - search_blocks, gridDim.x - search_blocks);
        return;
    }
    const Tables& T = *d.tab;
    // `split` workgroups share a chunk (small simulations, whose few chunks
    // would otherwise leave the claimers to a few workgroups): each compacts
    // the chunk and searches every split-th pass of its claimers
    // the chunks within the capacity are dealt to the XCDs; the chunks of
    // the slot headroom (holes beyond the capacity, rarely in use) come
    // last in dispatch order
    const uint32_t g = blockIdx.x < core_blocks ? xcd_chunk(core_blocks) : blockIdx.x;
    const uint32_t share = g % split;
    const uint32_t first = g / split * kPChunk;
    // The thread's four claimer flags, requested first.  The flag array is
    // padded to whole chunks and the grid covers the slots, so the word is
    // in bounds even past the live agents (whose count arrives with the
    // control block).
    const uint32_t word =
        *reinterpret_cast<const FlagWord*>(d.sclaim + first + uint32_t(kClaimPer) * threadIdx.x);
    // claimers among the binned agents; a step that keeps the binning
    // searches from every slot
    const uint32_t n = bin ? d.ctl->n_binned : d.ctl->s[p].n_slots;
    const uint32_t t = d.ctl->s[p].t;
    const uint32_t n_glob = d.link ? d.ctl->n_glob : 0u;
    if (first >= n) return;
    {
        // rows of the species in use, as words; the radii of the rules
        const uint32_t nw = uint32_t(T.ns) * (kMaxSpecies / 4);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&T.rule_of[0][0]);
        uint32_t* dst = reinterpret_cast<uint32_t*>(P.rule_of);
        for (uint32_t q = threadIdx.x; q < nw; q += kPropBlock) dst[q] = src[q];
        for (uint32_t q = threadIdx.x; q < uint32_t(T.nr); q += kPropBlock) P.r2[q] = T.rule[q].r2;
        for (uint32_t q = threadIdx.x; q < uint32_t(T.ns); q += kPropBlock) {
            P.r2max[q] = T.claim_r2max[q];
            P.rmax[q] = T.claim_rmax[q];
            P.dmax[q] = T.claim_dmax[q];
        }
        if (threadIdx.x == 0) {
            nprop = 0;
            count = 0;
        }
    }
    __syncthreads();
    const uint32_t last = first + kPChunk < n ? first + kPChunk : n;
    const Agents A = d.a[p ^ 1];
    __shared__ uint32_t n_wide;
    const uint32_t nl = compact_claimers(word, first, last, list, &count, &n_wide);
    const uint32_t nw = n_wide;
    // A group of lanes per claimer: `narrow` lanes (4 for the 8-cell
    // stencil, 16 for the 27-cell one, or the configured count if more)
    // and `wide` = max(16, narrow) for the claimers that search 27 cells
    // while the others search 8.  Groups are laid out wide claimers first
    // over the workgroup's lanes, pass after pass, so every group is
    // aligned to its width; `split` workgroups sharing a chunk take every
    // split-th pass.
    const uint32_t wmin = T.stencil8 ? 4u : 16u;
    const uint32_t narrow = d.prop_lanes > wmin ? d.prop_lanes : wmin;
    const uint32_t wide = narrow > 16u ? narrow : 16u;
    const uint32_t lanes = nw * wide + (nl - nw) * narrow;
    for (uint32_t v = share * kPropBlock + threadIdx.x; v - threadIdx.x < lanes; v += kPropBlock * split) {
        if (v >= lanes) continue;
        uint32_t q, width;
        const bool is_wide = v < nw * wide;
        if (is_wide) {
            q = v / wide;
            width = wide;
        } else {
            q = nw + (v - nw * wide) / narrow;
            width = narrow;
        }
        const int li = int(v & (width - 1u));
        const uint32_t j = list[q];
        const uint4 rj = A.rec[j];
        const uint32_t ida = A.id[j];
        if (B)
            per_sim(sim_of(rj.w), [&](uint32_t u) {
                search_claimer<true>(d, d.tab[u], P, A, t, j, rj, ida, li, int(width), int(wide),
                                     is_wide, moved, n_glob, plocal, &nprop, &d.ctl->n_prop[p]);
            });
        else
            search_claimer<false>(d, T, P, A, t, j, rj, ida, li, int(width), int(wide), is_wide,
                                  moved, n_glob, plocal, &nprop, &d.ctl->n_prop[p]);
    }
    // the workgroup's proposers join the step's proposer list (one global
    // atomic per workgroup that has any)
    __syncthreads();
    const uint32_t np = nprop < kPropLds ? nprop : kPropLds;
    if (np == 0) return;
    if (threadIdx.x == 0) pbase = atomicAdd(&d.ctl->n_prop[p], np);
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < np; q += kPropBlock) d.plist[pbase + q] = plocal[q];
}

// The search over the claimer list (single simulations in list mode): the
// regions' counts give the step's n claimers; every claimer gets a group of
// L lanes, the widest power of two from 16 to 64 with n x L within the
// grid's lanes (so sparse claimers in crowded cells are searched by whole
// waves), and the groups are dealt over the workgroups in turn.  The
// proposals join the step's list as in the chunked search.
__global__ void __launch_bounds__(kPropBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_propose_list(Dev d, int p, int bin, uint32_t moved, uint32_t search_blocks)
{
    __shared__ uint4 plocal[kPropLds];
    __shared__ PairLds P;
    __shared__ uint32_t rstart[kListRegions + 1];
    __shared__ uint32_t nprop, pbase;
    if (blockIdx.x >= search_blocks) {
        sort_birth_runs(d, p, blockIdx.x - search_blocks, gridDim.x - search_blocks);
        return;
    }
    static_assert(kListRegions == 64, "one lane per region in the first wave");
    if (threadIdx.x < kListRegions) {
        // first claimer of each region in the step's order: a wave prefix
        const uint32_t c = d.ccount[threadIdx.x * kListStride];
        uint32_t incl = c;
        const int lane = lane_id();
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        rstart[threadIdx.x + 1] = incl;
        if (threadIdx.x == 0) {
            rstart[0] = 0;
            nprop = 0;
        }
    }
    __syncthreads();
    const uint32_t n = rstart[kListRegions];
    const uint32_t per0 = kPropBlock / 64u;  // groups of 64 per workgroup
    if (blockIdx.x * per0 >= n) return;      // no claimer for this workgroup at any width
    const Tables& T = *d.tab;
    {
        const uint32_t nw = uint32_t(T.ns) * (kMaxSpecies / 4);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&T.rule_of[0][0]);
        uint32_t* dst = reinterpret_cast<uint32_t*>(P.rule_of);
        for (uint32_t q = threadIdx.x; q < nw; q += kPropBlock) dst[q] = src[q];
        for (uint32_t q = threadIdx.x; q < uint32_t(T.nr); q += kPropBlock) P.r2[q] = T.rule[q].r2;
        for (uint32_t q = threadIdx.x; q < uint32_t(T.ns); q += kPropBlock) {
            P.r2max[q] = T.claim_r2max[q];
            P.rmax[q] = T.claim_rmax[q];
            P.dmax[q] = T.claim_dmax[q];
        }
    }
    __syncthreads();
    const uint32_t t = d.ctl->s[p].t;
    const uint32_t n_glob = d.link ? d.ctl->n_glob : 0u;
    const Agents A = d.a[p ^ 1];
    uint32_t L = 64;
    while (L > 16 && uint64_t(n) * L > uint64_t(search_blocks) * kPropBlock) L >>= 1;
    const uint32_t per = kPropBlock / L;  // groups per workgroup
    const int li = int(threadIdx.x & (L - 1u));
    // every lane of a group takes the same claimers, so a group's shuffles
    // stay among lanes that run them together
    for (uint32_t q = blockIdx.x * per + threadIdx.x / L; q < n; q += search_blocks * per) {
        // the region holding claimer q: the last with rstart <= q (regions
        // before it may be empty; q < n keeps it below the end)
        uint32_t r = 0;
#pragma unroll
        for (uint32_t h = kListRegions / 2; h; h >>= 1)
            if (rstart[r + h] <= q) r += h;
        const uint32_t e = d.clist[r * d.clist_cap + (q - rstart[r])];
        const uint32_t j = e & ~kListWide;
        const uint4 rj = A.rec[j];
        const uint32_t ida = A.id[j];
        search_claimer<false, true>(d, T, P, A, t, j, rj, ida, li, int(L), int(L),
                                    (e & kListWide) != 0u, moved, n_glob, plocal, &nprop,
                                    &d.ctl->n_prop[p]);
    }
    __syncthreads();
    const uint32_t np = nprop < kPropLds ? nprop : kPropLds;
    if (np == 0) return;
    if (threadIdx.x == 0) pbase = atomicAdd(&d.ctl->n_prop[p], np);
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < np; q += kPropBlock) d.plist[pbase + q] = plocal[q];
}

// ---------------------------------------------------------------------------
// finish: O7 confirmation and O8 pair products (only the claimer of a
// confirmed pair writes, and of a mutual homotypic pair only the lower id).
// The proposer entry carries the rule and whether the target claims too, so
// a confirmation reads only the two slots and the target's id and proposal.
// Species are written as single bytes, leaving the flag bytes alone.  In a
// step that keeps the binning, finish also places the step's children (its
// whole grid) and does the bookkeeping (its first workgroup).
// ---------------------------------------------------------------------------
template <bool B>
__global__ void __launch_bounds__(kBlock) k_finish(Dev d, int p, int record, int bin)
{
    __shared__ uint32_t s_dead;
    const Tables& T = *d.tab;
    Ctl* ctl = d.ctl;
    const uint32_t prop_blocks = gridDim.x - 1;  // the last workgroup keeps the books
    // the thread's first proposer entry is requested with the list's length
    // (entries past it are stale but inside the list's capacity)
    uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    uint4 e = q < d.slots ? d.plist[q] : uint4{};
    const uint32_t np = ctl->n_prop[p];
    const uint32_t t = ctl->s[p].t;
    // the claimer list's counters start the next step at zero (this step's
    // search has read them)
    if (d.list_mode && blockIdx.x == prop_blocks && threadIdx.x < kListRegions)
        d.ccount[threadIdx.x * kListStride] = 0u;
    if (!bin) {
        // a step that keeps the binning places its children here (a few by
        // the last workgroup, many by all) and does its bookkeeping
        const uint32_t nb = min(ctl->n_births[p], d.capacity);
        const BirthSlots bs = birth_slots(d, ctl->s[p], false, nb);
        place_births<B>(d, p, d.a[p ^ 1], nb, bs, record, blockIdx.x, gridDim.x, prop_blocks);
        if (blockIdx.x == prop_blocks) bookkeeping<B>(d, p, false);
    }
    if (blockIdx.x == prop_blocks || blockIdx.x * kBlock >= np) return;
    if (threadIdx.x == 0) s_dead = 0;
    __syncthreads();
    const Agents A = d.a[p ^ 1];
    for (; q < np; q += prop_blocks * kBlock) {
        if (q >= blockIdx.x * kBlock + kBlock) e = d.plist[q];
        const uint32_t j = e.x, b = e.y, ida = e.z;
        const int rule = int(e.w & 0xFFu);
        const bool b_claims = (e.w & uint32_t(kBestClaimer)) != 0;
        // the slots, the target's id and proposal, requested together
        const uint32_t idb = A.id[b], pb = d.prop[b];
        const unsigned long long slot_j = d.slot[j], slot_b = d.slot[b];
        const uint32_t lo_id = ida < idb ? ida : idb, hi_id = ida < idb ? idb : ida;
        // the pair's simulation gives the Philox key
        const Tables& Tk = B ? d.tab[e.w >> 16] : T;
        const unsigned long long pr = (unsigned long long)draw(Tk, lo_id, t, kPrio, hi_id).w0 << 32;
        if (slot_j != (pr | idb) || slot_b != (pr | ida)) continue;
        // b proposed too only if it carries the claimer flag (its prop is
        // then this step's); a mutual pair fires once, from the lower id
        if (idb < ida && b_claims && pb == j) continue;
        const RuleDev& R = T.rule[rule];
        set_species(A, j, R.p0 < 0 ? kDead : uint32_t(R.p0));
        set_species(A, b, R.p1 < 0 ? kDead : uint32_t(R.p1));
        const uint32_t h = (R.p0 < 0 ? 1u : 0u) + (R.p1 < 0 ? 1u : 0u);
        if (h) {
            // removals of the pair's simulation (a single simulation's are
            // summed per workgroup first)
            if (B) atomicAdd(&d.sc.dead[p][e.w >> 16], h);
            else atomicAdd(&s_dead, h);
        }
        if (record) {
            d.rpartner[j] = idb;
            d.rpartner[b] = ida;
        }
    }
    __syncthreads();
    if (!B && threadIdx.x == 0 && s_dead) atomicAdd(&d.sc.dead[p][0], s_dead);
}

// per-species counts of live agents (LDS histogram, one atomic per species
// per workgroup)
__global__ void __launch_bounds__(kBlock) k_counts(Dev d, int cur)
{
    __shared__ uint32_t h[kMaxSpecies];
    if (threadIdx.x < kMaxSpecies) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = d.ctl->s[cur].n_slots;
    const uint4* rec = d.a[cur].rec;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint32_t s = rec[i].w & 0xFFu;
        if (s < uint32_t(kMaxSpecies)) atomicAdd(&h[s], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxSpecies && h[threadIdx.x])
        atomicAdd(&d.counts[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// per (simulation, species) counts of a batch: one workgroup per 256 slots,
// the LDS histogram holding the simulation of the workgroup's first slot and
// the next one (agents are sorted by simulation); any other goes to memory
__global__ void __launch_bounds__(kBlock) k_counts_batch(Dev d, int cur)
{
    __shared__ uint32_t h[2][kMaxSpecies];
    __shared__ uint32_t base;
    const uint32_t n = d.ctl->s[cur].n_slots;
    const uint32_t first = blockIdx.x * kBlock;
    if (first >= n) return;
    const uint4* rec = d.a[cur].rec;
    if (threadIdx.x < 2 * kMaxSpecies) h[threadIdx.x / kMaxSpecies][threadIdx.x % kMaxSpecies] = 0;
    if (threadIdx.x == 0) base = sim_of(rec[first].w);
    __syncthreads();
    const uint32_t i = first + threadIdx.x;
    if (i < n) {
        const uint32_t w = rec[i].w;
        const uint32_t s = w & 0xFFu, sim = sim_of(w);
        if (s < uint32_t(kMaxSpecies)) {
            if (sim - base < 2u) atomicAdd(&h[sim - base][s], 1u);
            else atomicAdd(&d.counts[size_t(sim) * kMaxSpecies + s], 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMaxSpecies) {
        const uint32_t k = threadIdx.x / kMaxSpecies, s = threadIdx.x % kMaxSpecies;
        if (h[k][s] && base + k < d.n_sims)
            atomicAdd(&d.counts[size_t(base + k) * kMaxSpecies + s], (unsigned long long)h[k][s]);
    }
}

// State digest (verification only): each live agent contributes a 64-bit
// hash of (id, species, position bits), mixed by the finaliser of Appleby's
// MurmurHash3, and a simulation's digest is the sum of its agents' hashes
// mod 2^64, so it does not depend on where the agents sit in the arrays.
// Each wave walks a contiguous run of slots, sums its lanes per simulation
// (agents are sorted by simulation, so a run meets few) and adds each
// simulation's partial sum with one atomic when the simulation changes.
__device__ __forceinline__ uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDull;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint64_t agent_hash(uint32_t id, const uint4& r)
{
    uint64_t v = fmix64(((uint64_t(id) << 32) | (r.w & 0xFFu)) ^ 0x9E3779B97F4A7C15ull);
    v = fmix64(v ^ ((uint64_t(r.x) << 32) | r.y));
    return fmix64(v ^ uint64_t(r.z));
}

__global__ void __launch_bounds__(kBlock) k_digest(Dev d, int cur, unsigned long long* out,
                                                   uint32_t per_wave)
{
    const uint32_t n = d.ctl->s[cur].n_slots;
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t lo = wave * per_wave;
    const uint32_t hi = lo + per_wave < n ? lo + per_wave : n;
    const Agents A = d.a[cur];
    uint32_t acc_sim = kNone;  // wave-uniform
    unsigned long long acc = 0;
    for (uint32_t base = lo; base < hi; base += 64) {
        const uint32_t i = base + uint32_t(lane_id());
        uint32_t sim = kNone;
        unsigned long long h = 0;
        if (i < hi) {
            const uint4 r = A.rec[i];
            if ((r.w & 0xFFu) != kDead) {
                sim = sim_of(r.w);
                h = agent_hash(A.id[i], r);
            }
        }
        // per simulation present in this round of lanes, in lane order
        uint64_t left = __ballot(sim != kNone);
        while (left) {
            const uint32_t u = __shfl(sim, __builtin_ctzll(left), 64);
            unsigned long long v = sim == u ? h : 0ull;
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (u != acc_sim) {
                if (acc_sim != kNone && lane_id() == 0) atomicAdd(&out[acc_sim], acc);
                acc_sim = u;
                acc = 0;
            }
            acc += v;
            left &= ~__ballot(sim == u);
        }
    }
    if (acc_sim != kNone && lane_id() == 0) atomicAdd(&out[acc_sim], acc);
}

// Gathers simulation `sim`'s live agents (queries between steps): the
// record and id of each go to the birth records, its recorded cell id and
// partner to bkey and its recorded event to `event`, at an index from one
// atomic per wave; ctl->export_n counts them (cleared by the caller).
__global__ void __launch_bounds__(kBlock) k_export(Dev d, int cur, uint32_t sim, int record)
{
    const uint32_t n = d.ctl->s[cur].n_slots;
    const Agents A = d.a[cur];
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; (i & ~63u) < n; i += stride) {
        uint4 r = {0u, 0u, 0u, kDead};
        if (i < n) r = A.rec[i];
        const bool mine = (r.w & 0xFFu) != kDead && sim_of(r.w) == sim;
        const uint32_t k = wave_append(&d.ctl->export_n, mine);
        if (!mine || k >= d.capacity) continue;
        d.births[k] = Birth{A.id[i], r.w, __uint_as_float(r.x), __uint_as_float(r.y),
                            __uint_as_float(r.z)};
        if (record) {
            d.bkey[k] = ((unsigned long long)d.rkey[i] << 32) | d.rpartner[i];
            d.event[k] = d.revent[i];
        }
    }
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// clears the counts; a counts-ring entry also gets the step counter
__global__ void k_zero_counts(Dev d, int cur, unsigned long long* tslot)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < d.n_sims * uint32_t(kMaxSpecies)) d.counts[i] = 0ull;
    if (tslot && i == 0) *tslot = d.ctl->s[cur].t;
}

}  // namespace

// ---------------------------------------------------------------------------
// launch entry points.  Agent-indexed kernels are sized for the capacity and
// read the live sizes from the control block, so a step needs no host
// synchronisation and can be captured in a graph.
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(uint32_t n) { return n ? (n + kBlock - 1) / kBlock : 1u; }
static constexpr unsigned kFinishBlocks = 64;
static constexpr unsigned kPropMinBlocks = 2048;  // default fewest propose workgroups
static inline unsigned chunks_for(uint32_t n) { return n ? (n + kPChunk - 1) / kPChunk : 1u; }

void launch_init(const Dev& d, hipStream_t s)
{
    if (d.n_init) k_init<<<blocks_for(d.n_init), kBlock, 0, s>>>(d);
}
void launch_fill_records(const Dev& d, hipStream_t s)
{
    k_fill_records<<<blocks_for(d.slots), kBlock, 0, s>>>(d);
    const uint32_t cells = (d.ntiles << (kScanTileLog + d.tile_shift)) + 1u;
    k_fill_heads<<<blocks_for(cells), kBlock, 0, s>>>(d, cells);
}
template <class K, class... Args>
static inline void go(K kernel, unsigned grid, unsigned block, hipStream_t s, const KEvents& ev,
                      Args... args)
{
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, ev.start, ev.stop, 0, args...);
}

// the batch variants of the agent kernels (template argument true) resolve
// each agent's simulation; a single simulation takes the plain ones
void launch_move(const Dev& d, int p, int record, int bin, uint32_t moved, hipStream_t s,
                 const KEvents& ev)
{
    if (d.n_sims > 1)
        go(k_move<true>, blocks_for(d.span), kBlock, s, ev, d, p, record, bin, moved);
    else go(k_move<false>, blocks_for(d.span), kBlock, s, ev, d, p, record, bin, moved);
}

void launch_scan(const Dev& d, int p, hipStream_t s, const KEvents& ev)
{
    // the tiles, then the birth-run sorters (models that place children)
    go(k_scan, d.ntiles + d.birth_blocks, kScanThreads, s, ev, d, p);
}
void launch_scatter(const Dev& d, int p, int record, hipStream_t s, const KEvents& ev)
{
    // one workgroup per 256 slots, then the workgroups that place the
    // children (at least one: it also does the bookkeeping)
    const unsigned agents = blocks_for(d.span);
    const unsigned grid = agents + (d.birth_blocks ? d.birth_blocks : 1u);
    if (d.n_sims > 1) go(k_scatter<true>, grid, kBlock, s, ev, d, p, record, agents);
    else go(k_scatter<false>, grid, kBlock, s, ev, d, p, record, agents);
}
void launch_propose(const Dev& d, int p, int bin, uint32_t moved, hipStream_t s, const KEvents& ev)
{
    // enough workgroups to fill the chip: chunks shared by up to 16
    const unsigned chunks = chunks_for(d.span);
    unsigned split = 1;
    const unsigned min_blocks = d.prop_min_blocks ? d.prop_min_blocks : kPropMinBlocks;
    while (split < 16 && chunks * split * 2 <= min_blocks) split *= 2;
    // a step that keeps the binning sorts its birth runs in extra workgroups
    const unsigned search = chunks * split;
    const unsigned core = chunks_for(d.capacity) * split;
    const unsigned grid = search + (bin ? 0u : d.birth_blocks);
    if (d.list_mode) {
        go(k_propose_list, d.list_blocks + (bin ? 0u : d.birth_blocks), kPropBlock, s, ev, d, p,
           bin, moved, d.list_blocks);
        return;
    }
    if (d.n_sims > 1)
        go(k_propose<true>, grid, kPropBlock, s, ev, d, p, split, bin, moved, search, core);
    else go(k_propose<false>, grid, kPropBlock, s, ev, d, p, split, bin, moved, search, core);
}
void launch_finish(const Dev& d, int p, int record, int bin, hipStream_t s, const KEvents& ev)
{
    // a fixed grid strides over the step's proposer list (and a kept step's
    // children), and one more workgroup keeps the books
    unsigned nb = blocks_for(d.capacity);
    if (nb > kFinishBlocks) nb = kFinishBlocks;
    nb += 1;
    if (d.n_sims > 1) go(k_finish<true>, nb, kBlock, s, ev, d, p, record, bin);
    else go(k_finish<false>, nb, kBlock, s, ev, d, p, record, bin);
}
void launch_digest(const Dev& d, int cur, unsigned long long* out, hipStream_t s)
{
    k_zero_u64<<<blocks_for(d.n_sims), kBlock, 0, s>>>(out, d.n_sims);
    // about 4,096 waves, each over a whole number of 64-slot rounds
    const uint32_t waves = 4096;
    uint32_t per_wave = (d.slots + waves - 1) / waves;
    per_wave = (per_wave + 63u) / 64u * 64u;
    const uint32_t need = (d.slots + per_wave - 1) / per_wave;  // waves that have slots
    k_digest<<<(need + 3) / 4, kBlock, 0, s>>>(d, cur, out, per_wave);
}

void launch_export(const Dev& d, int cur, uint32_t sim, int record, hipStream_t s)
{
    unsigned nb = blocks_for(d.slots);
    if (nb > 4096) nb = 4096;
    k_export<<<nb, kBlock, 0, s>>>(d, cur, sim, record);
}

void launch_counts(const Dev& d0, int cur, hipStream_t s, unsigned long long* dst,
                   unsigned long long* tslot)
{
    Dev d = d0;
    if (dst) d.counts = dst;
    k_zero_counts<<<blocks_for(d.n_sims * uint32_t(kMaxSpecies)), kBlock, 0, s>>>(d, cur, tslot);
    if (d.n_sims > 1) {
        k_counts_batch<<<blocks_for(d.slots), kBlock, 0, s>>>(d, cur);
        return;
    }
    unsigned nb = blocks_for(d.slots);
    if (nb > 2048) nb = 2048;
    k_counts<<<nb, kBlock, 0, s>>>(d, cur);
}

}  // namespace mabm
