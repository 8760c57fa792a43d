// api.hip -- host engine behind the C ABI of include/mabm.h: model
// validation, arena carving, table construction, step sequencing on the
// caller's stream, synchronising queries and per-kernel event timing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mabm.h"
#include "engine.hpp"

using namespace mabm;

namespace {

struct SpeciesHost {
    std::string name;
    float D;
    uint32_t count;
    int32_t comp;
};

struct EventPair {
    hipEvent_t a, b;
};

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

float extent_of(const mabm_config& c)
{
    return c.geometry == MABM_PERIODIC_BOX ? c.box_um : c.outer_radius_um * 2.0f;
}

constexpr uint32_t kMaxGrid = MABM_MAX_GRID;  // cells per axis (10-bit Morton coordinates)
// cells of all simulations together: cell keys, cell-table indices and the
// counting sort's prefix sums are 32-bit words
constexpr uint64_t kMaxCells = 1ull << 31;
static_assert(kMaxGrid <= 1024, "Morton keys interleave 10-bit cell coordinates");

// cells per axis implied by the configuration alone: the requested cell
// size, or the power of two nearest (in log) to one cell per agent of
// capacity over the bounding box
uint32_t grid_from_config(const mabm_config& c)
{
    const double ext = extent_of(c);
    double g;
    if (c.cell_um > 0.0f) g = std::floor(ext / (double)c.cell_um);
    else g = std::exp2(std::round(std::log2(std::cbrt((double)c.capacity))));
    return (uint32_t)std::min((double)kMaxGrid, std::max(3.0, g));
}

// bits per axis of the Morton sort key for G cells per axis
uint32_t morton_bits(uint32_t g)
{
    uint32_t b = 0;
    while ((1u << b) < g) ++b;
    return b;
}

bool config_ok(const mabm_config* c, std::string& why)
{
    if (!c) { why = "null config"; return false; }
    if (c->abi_version != MABM_ABI_VERSION) { why = "abi_version mismatch"; return false; }
    if (c->geometry < 0 || c->geometry > 2) { why = "bad geometry"; return false; }
    if (c->geometry == MABM_PERIODIC_BOX && !(c->box_um > 0.0f)) { why = "box_um must be > 0"; return false; }
    if (c->geometry != MABM_PERIODIC_BOX && !(c->outer_radius_um > 0.0f)) { why = "outer_radius_um must be > 0"; return false; }
    if (c->geometry == MABM_NESTED_SPHERES &&
        !(c->inner_radius_um > 0.0f && c->inner_radius_um < c->outer_radius_um)) {
        why = "need 0 < inner_radius_um < outer_radius_um";
        return false;
    }
    if (!(c->dt_s > 0.0f)) { why = "dt_s must be > 0"; return false; }
    // (slot indices then stay below the extra-chain markers)
    static_assert((1u << 30) < kUnlinked, "slot indices below the chain markers");
    if (c->capacity == 0 || c->capacity > (1u << 30)) { why = "capacity must be in [1, 2^30]"; return false; }
    static_assert((1u << 30) + (1u << 28) + 1024 < kUnlinked, "slots of 2^30 agents below the chain markers");
    if (c->cell_um < 0.0f) { why = "cell_um must be >= 0"; return false; }
    return true;
}

// Per-simulation counters, kSimWords arrays of n_sims words in the arena, in
// this order: live, dead[0], dead[1], born[0], born[1], next_id[0],
// next_id[1] (SimCounters).
constexpr int kSimWords = 7;

// Arena layout: every array 256-byte aligned, in this order.
struct Layout {
    size_t ctl, tab, rec[2], id[2], rank, event, sclaim, cell_count, cell_start, tile_acc, slot,
        prop, plist, rkey, revent, rpartner, births, bkey, brank, hlist, counts, digest, simc,
        head, nxt, glob, total;
    uint32_t ncells, ntiles, tile_shift, clist_cap;
    size_t clist, ccount;
    uint32_t capacity, slots;
};

// Entries of the agent arrays for a summed capacity: the capacity plus a
// quarter for holes.  Agents that a step removes occupy their slots until a
// binning drops them, or until a child of a later step that keeps the
// binning takes the slot over; a step's children go after the slots in
// use.  The slots in use therefore stay within the live agents plus the
// removals of a single step's pair rules, and the headroom covers removals
// of up to a quarter of the capacity in one step.
uint64_t slots_for(uint64_t capacity) { return capacity + capacity / 4 + 1024; }

// Layout of one simulation (n = 1) or of a batch of n: agent arrays sized
// for the summed capacities, the simulations' cell grids one after another
// (each at most 8^bits of its configured grid; a contact radius can only
// coarsen it), one table set and one id counter per simulation.
Layout make_layout(const mabm_config* cs, uint32_t n)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    size_t cap = 0, cells = 0;
    for (uint32_t k = 0; k < n; ++k) {
        cap += cs[k].capacity;
        cells += (size_t)1 << (3 * morton_bits(grid_from_config(cs[k])));
    }
    const size_t births = cap;  // a parent has at most one child per step
    L.capacity = (uint32_t)cap;
    L.slots = (uint32_t)slots_for(cap);
    cap = L.slots;  // every per-slot array
    L.ncells = (uint32_t)cells;
    L.tile_shift = 0;
    while (((cells + ((size_t)kScanTile << L.tile_shift) - 1) >> (kScanTileLog + L.tile_shift)) >
           kMaxScanTiles)
        ++L.tile_shift;
    L.ntiles = (uint32_t)((cells + ((size_t)kScanTile << L.tile_shift) - 1) >> (kScanTileLog + L.tile_shift));
    L.ctl = take(sizeof(Ctl));
    L.tab = take(sizeof(Tables) * n);
    for (int b = 0; b < 2; ++b) {
        L.rec[b] = take(cap * 16);
        L.id[b] = take(cap * 4);
    }
    L.rank = take(cap * 4);
    L.event = take(cap);
    L.sclaim = take((cap + kClaimChunk - 1) / kClaimChunk * kClaimChunk);  // whole chunks
    const size_t padded = (size_t)L.ntiles << (kScanTileLog + L.tile_shift);  // whole scan tiles
    L.cell_count = take(padded * 4);
    L.cell_start = take((padded + 1) * 4);
    L.tile_acc = take((size_t)2 * L.ntiles * kTileStride * 4);
    L.slot = take(cap * 8);
    L.prop = take(cap * 4);
    L.plist = take(cap * 16);
    L.rkey = take(cap * 4);
    L.revent = take(cap);
    L.rpartner = take(cap * 4);
    L.births = take(births * sizeof(Birth));
    L.bkey = take(births * 8);
    L.brank = take(births * 8);
    L.hlist = take(cap * 4);
    L.counts = take((size_t)kMaxSpecies * 8 * n);
    L.digest = take((size_t)8 * n);
    L.simc = take((size_t)4 * kSimWords * n);
    L.head = take((padded + 1) * 4);
    L.nxt = take(cap * 4);
    L.glob = take(cap * 4);
    // claimer list: each region takes the claimers of every kListRegions-th
    // workgroup of move or scatter (one agent slot per thread)
    const size_t wgs = (cap + 255) / 256;
    L.clist_cap = (uint32_t)((wgs + kListRegions - 1) / kListRegions * 256);
    L.clist = take((size_t)kListRegions * L.clist_cap * 4);
    L.ccount = take((size_t)kListRegions * kListStride * 4);
    L.total = off;
    return L;
}

// total capacity of a batch, 0 if it does not fit the 32-bit slot indices
uint64_t total_capacity(const mabm_config* cs, uint32_t n)
{
    uint64_t cap = 0;
    for (uint32_t k = 0; k < n; ++k) cap += cs[k].capacity;
    return cap;
}

uint64_t threshold_of(double p)
{
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)std::floor(p * 4294967296.0);
}

}  // namespace

struct mabm_sim {
    mabm_config cfg{};                 // the first simulation's configuration
    std::vector<mabm_config> cfgs;     // one per simulation (a single one: {cfg})
    uint32_t n_sims = 1;
    std::vector<std::vector<uint32_t>> sim_counts;  // [species][simulation] initial counts
    std::vector<Tables> tabs;          // one per simulation
    std::vector<uint32_t> sim_G;
    std::vector<float> sim_h;
    std::vector<uint32_t> host_simc;     // staging for the per-simulation counters
    uint64_t steps_done = 0;             // steps enqueued since finalize
    // counts ring (caller's device memory): entries of ring_words u64
    unsigned long long* ring = nullptr;
    uint32_t ring_entries = 0, ring_every = 0;
    uint64_t ring_recorded = 0;
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    Layout lay{};
    Dev dev{};
    std::vector<SpeciesHost> species;
    std::vector<mabm_rule> rules;
    bool finalized = false, failed = false, has_bimol = false;
    int static_device = -1;  // device whose static arena holds this simulation (-1: none)
    // captured steps (one step, and graph_steps steps) per starting state:
    // parity, agent buffer and steps since the last binning
    std::map<uint32_t, hipGraphExec_t> graphs;
    int parity = 0;
    // Binning schedule: the cell lists are rebuilt every `bin_every` steps
    // (1: every step); `buf` is the agent buffer holding the current state,
    // `kept` the steps since the last binning (bin_every - 1 forces one)
    uint32_t bin_every = 1, bin_every_max = 0, kept = 0;
    uint32_t propose_mode = 0;  // MABM_PARAM_PROPOSE_MODE as set (0: auto)
    int buf = 0;
    uint32_t G = 0;
    float h = 0.0f;
    std::string err;
    // per-kernel timing
    bool prof = false;
    std::vector<EventPair> pool;
    std::vector<int> pending_kernel;
    size_t pending = 0;
    uint64_t launches[kNumKernels] = {};
    double total_ms[kNumKernels] = {};
};

namespace {

mabm_status fail(mabm_sim* s, mabm_status code, const std::string& msg)
{
    s->err = msg;
    return code;
}

// u64 words of a counts-ring entry: the step counter, then the counts of
// every (simulation, species) pair, kMaxSpecies per simulation
size_t ring_words(const mabm_sim* s) { return 1 + (size_t)s->n_sims * kMaxSpecies; }

bool is_batch(mabm_sim* s, const char* call)
{
    if (s->n_sims == 1) return false;
    s->err = std::string(call) + " refers to one simulation; this handle holds a batch";
    return true;
}

mabm_status hip_fail(mabm_sim* s, hipError_t e, const char* what)
{
    s->failed = true;
    return fail(s, MABM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OK(sim, call)                                 \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(sim, e_, #call); \
    } while (0)

// harvest finished timing events (blocking on them)
void harvest(mabm_sim* s)
{
    for (size_t k = 0; k < s->pending; ++k) {
        EventPair& p = s->pool[k];
        (void)hipEventSynchronize(p.b);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            s->total_ms[s->pending_kernel[k]] += ms;
            s->launches[s->pending_kernel[k]] += 1;
        }
    }
    s->pending = 0;
}

// Launch one step kernel; with timing on, its dispatch stamps a pooled
// event pair at the kernel's start and end.
template <class F>
void timed(mabm_sim* s, int kid, F&& launch)
{
    if (!s->prof) {
        launch(KEvents{});
        return;
    }
    if (s->pending == s->pool.size()) harvest(s);
    EventPair& p = s->pool[s->pending];
    s->pending_kernel[s->pending] = kid;
    ++s->pending;
    launch(KEvents{p.a, p.b});
}

// Steps between binnings.  Between two binnings the agents keep their slots
// and the neighbour search reads the cell lists of the last binning, in
// which an agent may lie up to j moves away from where it now is.  A step's
// move along an axis is sigma |z| with |z| < sqrt(-2 ln 2^-24) = 5.768 (the
// smallest uniform the Box-Muller draw takes is 2^-24; 5.78 leaves room for
// the approximations of log and cosine), sigma being that of the agent's
// species at the time, so a target of a claimer's rules moves at most
// claim_dmax per step (the largest bound over every species that is, or can
// turn into, such a target).  While a claimer species' largest contact
// radius plus j such moves stays within its stencil's reach (half a cell
// for the 8-cell stencil, a whole cell for the 27-cell one, less 1 %),
// every partner within reach is still found and the results are those of
// binning every step; a claimer species whose reach outgrows the 8-cell
// stencil searches 27 cells in the later kept steps.  Agents that rules
// place (newborns, translocated agents, split parents) are far from any
// cell list: while a binning is kept they join extra per-cell chains at
// their new positions (or, placed twice, a global list), which the search
// reads too.  Models without pair rules bin every step (nothing searches).
constexpr uint32_t kMaxBinEvery = 8;
constexpr uint32_t kModeChunks = 1, kModeList = 2;  // MABM_PARAM_PROPOSE_MODE values
constexpr uint32_t kListBlocks = 2048;              // workgroups of the claimer-list search
constexpr double kNormalBound = 5.78;

// whether the model allows keeping cell lists at all: it has pair rules
// (else nothing searches them)
bool may_keep_binning(const mabm_sim* s)
{
    for (const mabm_rule& u : s->rules)
        if (u.kind == MABM_BIMOL) return true;
    return false;
}

// whether the model has rules with children (splits, emissions)
bool has_births(const mabm_sim* s)
{
    for (const mabm_rule& u : s->rules)
        if (u.kind == MABM_UNIMOL && (u.placement == MABM_SPLIT || u.placement == MABM_EMIT))
            return true;
    return false;
}

// whether the model has rules that place agents (births, translocations)
bool places_agents(const mabm_sim* s)
{
    for (const mabm_rule& u : s->rules)
        if (u.kind == MABM_UNIMOL && u.placement != MABM_KEEP) return true;
    return false;
}

// tables of simulation k of s (the only one, or one of a batch)
mabm_status build_one(mabm_sim* s, uint32_t k_sim, Tables& T)
{
    std::memset(&T, 0, sizeof T);
    const mabm_config& c = s->cfgs[k_sim];
    const int ns = (int)s->species.size(), nr = (int)s->rules.size();
    if (ns == 0) return fail(s, MABM_E_INVALID, "no species");
    T.geometry = c.geometry;
    T.ncomp = c.geometry == MABM_NESTED_SPHERES ? 2 : 1;
    T.ns = ns;
    T.nr = nr;
    T.L = c.box_um;
    T.halfL = c.box_um * 0.5f;
    T.Rout = c.outer_radius_um;
    T.Rin = c.inner_radius_um;
    T.Rout2 = (float)((double)c.outer_radius_um * (double)c.outer_radius_um);
    T.Rin2 = (float)((double)c.inner_radius_um * (double)c.inner_radius_um);
    T.key0 = (uint32_t)c.seed;
    T.key1 = (uint32_t)(c.seed >> 32);
    T.capacity = c.capacity;
    uint64_t acc = 0;
    for (int k = 0; k < ns; ++k) {
        acc += s->sim_counts[k][k_sim];
        T.init_end[k] = (uint32_t)acc;
        T.init_comp[k] = s->species[k].comp;
        T.sigma[k] = (float)std::sqrt(2.0 * (double)s->species[k].D * (double)c.dt_s);
    }
    if (acc > c.capacity) return fail(s, MABM_E_CAPACITY, "initial counts exceed the capacity");
    // species x can become species y (the same agent): through a
    // conversion, or as a pair rule's claimer or target product
    bool becomes[kMaxSpecies][kMaxSpecies] = {};
    for (int k = 0; k < ns; ++k) becomes[k][k] = true;
    for (const mabm_rule& u : s->rules) {
        if (u.reactant[0] >= 0 && u.product[0] >= 0) becomes[u.reactant[0]][u.product[0]] = true;
        if (u.kind == MABM_BIMOL && u.reactant[1] >= 0 && u.product[1] >= 0)
            becomes[u.reactant[1]][u.product[1]] = true;
    }
    for (int m = 0; m < ns; ++m)
        for (int a = 0; a < ns; ++a)
            for (int b = 0; b < ns; ++b)
                if (becomes[a][m] && becomes[m][b]) becomes[a][b] = true;
    for (int a = 0; a < kMaxSpecies; ++a)
        for (int b = 0; b < kMaxSpecies; ++b) T.rule_of[a][b] = kNoRule;
    double rmax = 0.0;
    s->has_bimol = false;
    for (int r = 0; r < nr; ++r) {
        const mabm_rule& u = s->rules[r];
        RuleDev& R = T.rule[r];
        R.kind = u.kind;
        R.placement = u.placement;
        R.p0 = u.product[0];
        R.p1 = u.product[1];
        R.to = u.to_comp;
        R.r2 = (float)((double)u.radius_um * (double)u.radius_um);
        R.release = u.release_radius_um;
        R.release2 = (float)((double)u.release_radius_um * (double)u.release_radius_um);
        R.thr = threshold_of(u.prob_per_step);
        if (u.placement == MABM_TRANSLOCATE)
            R.target_r = (float)(u.to_comp == 0 ? (double)c.inner_radius_um - (double)u.release_radius_um
                                                : (double)c.inner_radius_um + (double)u.release_radius_um);
        if (u.kind == MABM_BIMOL) {
            T.rule_of[u.reactant[0]][u.reactant[1]] = (uint8_t)r;
            T.claimer[u.reactant[0]] = 1;
            T.claim_r2max[u.reactant[0]] = std::max(T.claim_r2max[u.reactant[0]], R.r2);
            T.claim_rmax[u.reactant[0]] = std::max(T.claim_rmax[u.reactant[0]], u.radius_um);
            for (int k = 0; k < ns; ++k)
                if (becomes[k][u.reactant[1]])
                    T.claim_dmax[u.reactant[0]] =
                        std::max(T.claim_dmax[u.reactant[0]], (float)(kNormalBound * (double)T.sigma[k]));
            rmax = std::max(rmax, (double)u.radius_um);
            s->has_bimol = true;
        }
    }
    // unimolecular cumulative thresholds per (species, compartment), rule-id order
    for (int k = 0; k < ns; ++k)
        for (int cc = 0; cc < T.ncomp; ++cc) {
            double cum = 0.0;
            for (int r = 0; r < nr; ++r) {
                const mabm_rule& u = s->rules[r];
                if (u.kind != MABM_UNIMOL || u.reactant[0] != k) continue;
                if (u.from_comp != -1 && u.from_comp != cc) continue;
                if (T.uni_n[k][cc] >= kMaxUni)
                    return fail(s, MABM_E_INVALID, "more than 8 unimolecular rules for one species");
                cum += u.prob_per_step;
                if (cum > 1.0)
                    return fail(s, MABM_E_INVALID,
                                "unimolecular probabilities of a species sum above 1");
                const int j = T.uni_n[k][cc]++;
                T.uni_rule[k][cc][j] = (uint8_t)r;
                T.uni_thr[k][cc][j] = threshold_of(cum);
            }
        }
    // move's per-(species, compartment) digest of the tables above
    for (int k = 0; k < ns; ++k)
        for (int cc = 0; cc < 2; ++cc) {
            SpecHot& H = T.hot[k][cc];
            H.sigma = T.sigma[k];
            H.rmax = T.claim_rmax[k];
            H.dmax = T.claim_dmax[k];
            H.claimer = T.claimer[k];
            H.uni_n = T.uni_n[k][cc];
            if (H.uni_n) {
                H.rule0 = T.uni_rule[k][cc][0];
                H.always = T.uni_thr[k][cc][0] >= (1ull << 32) ? 1 : 0;
                H.thr0 = H.always ? 0u : (uint32_t)T.uni_thr[k][cc][0];
            }
        }
    // spatial hash: G cells per axis, cell size >= 1.01 R_max
    const double ext = extent_of(c);
    uint32_t G = grid_from_config(c);
    // Default grid: the power of two nearest (in log) to cells holding two
    // of the initial agents on average over the volume they fill, if that is
    // coarser than the arena's grid (sized from the capacity, which counts
    // room for births, over the whole bounding box).  A search costs little
    // more at a few agents per cell while the cell tables, which the
    // counting sort scans at every binning, shrink with the cube of the cell.
    if (c.cell_um <= 0.0f && acc > 0) {
        const double pi = 3.14159265358979323846;
        const double vol = c.geometry == MABM_PERIODIC_BOX
                               ? ext * ext * ext
                               : 4.0 / 3.0 * pi * std::pow((double)c.outer_radius_um, 3.0);
        const double h = std::cbrt(2.0 * vol / (double)acc);
        const double g = std::exp2(std::round(std::log2(ext / h)));
        G = std::min(G, (uint32_t)std::min((double)kMaxGrid, std::max(3.0, g)));
    }
    if (rmax > 0.0 && ext / G < 1.01 * rmax) {
        if (c.cell_um > 0.0f)
            return fail(s, MABM_E_INVALID, "cell_um smaller than 1.01 x the largest contact radius");
        G = (uint32_t)std::floor(ext / (1.01 * rmax));
        if (G < 3) return fail(s, MABM_E_INVALID, "volume smaller than 3 cells of the contact radius");
    }
    s->sim_G[k_sim] = G;
    s->sim_h[k_sim] = (float)(ext / G);
    T.G = G;
    T.morton_bits = morton_bits(G);
    T.lo = c.geometry == MABM_PERIODIC_BOX ? 0.0f : -c.outer_radius_um;
    T.inv_h = (float)((double)G / ext);
    T.stencil8 = (rmax > 0.0 && ext / G >= 2.02 * rmax) ? 1u : 0u;
    return MABM_OK;
}

// every simulation's tables, and their places in the batch: cells and
// initial slots one simulation after another; the 8-cell stencil only if
// every simulation allows it (the search then has one lane layout)
mabm_status build_tables(mabm_sim* s)
{
    const uint32_t n = s->n_sims;
    s->tabs.assign(n, Tables{});
    s->sim_G.assign(n, 0u);
    s->sim_h.assign(n, 0.0f);
    uint64_t cell_base = 0, slot_base = 0;
    uint32_t stencil8 = 1;
    for (uint32_t k = 0; k < n; ++k) {
        Tables& T = s->tabs[k];
        mabm_status st = build_one(s, k, T);
        if (st != MABM_OK) return st;
        T.sim = k;
        T.cell_base = (uint32_t)cell_base;
        T.slot_base = (uint32_t)slot_base;
        cell_base += (uint64_t)1 << (3 * T.morton_bits);
        slot_base += T.init_end[T.ns - 1];
        stencil8 &= T.stencil8;
    }
    for (Tables& T : s->tabs) T.stencil8 = stencil8;
    s->G = s->sim_G[0];
    s->h = s->sim_h[0];
    return MABM_OK;
}

// whether claimer species sp needs the 27-cell stencil in some step of a
// binning kept for k steps, in any simulation
bool needs_wide(const mabm_sim* s, int sp, uint32_t k)
{
    for (uint32_t m = 0; m < s->n_sims; ++m) {
        const Tables& T = s->tabs[m];
        const double req = (double)T.claim_rmax[sp] + (double)(k - 1) * (double)T.claim_dmax[sp];
        if (!T.stencil8 || req > 0.5 * 0.99 * (double)s->sim_h[m]) return true;
    }
    return false;
}

void set_schedule(mabm_sim* s)
{
    uint32_t k = s->bin_every_max ? s->bin_every_max : kMaxBinEvery;
    if (!may_keep_binning(s)) k = 1;
    const Tables& T0 = s->tabs[0];
    // every claimer species' reach within the 27-cell stencil's
    for (uint32_t m = 0; m < s->n_sims; ++m)
        for (int sp = 0; sp < T0.ns; ++sp) {
            const double dmax = T0.claim_dmax[sp];
            if (!T0.claimer[sp] || dmax <= 0.0) continue;
            const double room = std::floor((0.99 * (double)s->sim_h[m] - (double)T0.claim_rmax[sp]) / dmax);
            k = (uint32_t)std::min((double)k, 1.0 + std::max(0.0, room));
        }
    // A claimer searches about three times the cells with the 27-cell
    // stencil: where the grid allows the 8-cell one, keep a binning longer
    // only while the claimer species that would need 27 cells hold at most
    // an eighth of the initial claimers.
    if (T0.stencil8) {
        while (k > 1) {
            uint64_t all = 0, wide = 0;
            for (int sp = 0; sp < T0.ns; ++sp) {
                if (!T0.claimer[sp]) continue;
                uint64_t n = 0;
                for (uint32_t m = 0; m < s->n_sims; ++m) n += s->sim_counts[sp][m];
                all += n;
                if (needs_wide(s, sp, k)) wide += n;
            }
            if (8 * wide <= all) break;
            --k;
        }
    }
    s->bin_every = std::max(1u, k);
    s->kept = s->bin_every - 1;  // the next step bins
    s->dev.link = s->bin_every > 1 && places_agents(s) ? 1u : 0u;
}

// whether the next step bins, given the steps kept since the last binning
bool bins(const mabm_sim* s, uint32_t kept) { return kept + 1 >= s->bin_every; }

// the device view of the current state (a[parity] = the buffer holding it)
Dev state_dev(const mabm_sim* s)
{
    Dev d = s->dev;
    d.a[s->parity] = s->dev.a[s->buf];
    return d;
}

void drop_graphs(mabm_sim* s)
{
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
}

void fill_dev(mabm_sim* s)
{
    Dev& d = s->dev;
    const Layout& L = s->lay;
    uint8_t* A = s->arena;
    d.ctl = (Ctl*)(A + L.ctl);
    d.tab = (const Tables*)(A + L.tab);
    for (int b = 0; b < 2; ++b) {
        d.a[b].rec = (uint4*)(A + L.rec[b]);
        d.a[b].id = (uint32_t*)(A + L.id[b]);
    }
    d.rank = (uint32_t*)(A + L.rank);
    d.event = A + L.event;
    d.sclaim = A + L.sclaim;
    d.cell_count = (uint32_t*)(A + L.cell_count);
    d.cell_start = (uint32_t*)(A + L.cell_start);
    d.tile_acc = (uint32_t*)(A + L.tile_acc);
    d.slot = (unsigned long long*)(A + L.slot);
    d.prop = (uint32_t*)(A + L.prop);
    d.plist = (uint4*)(A + L.plist);
    d.rkey = (uint32_t*)(A + L.rkey);
    d.revent = A + L.revent;
    d.rpartner = (uint32_t*)(A + L.rpartner);
    d.births = (Birth*)(A + L.births);
    d.bkey = (unsigned long long*)(A + L.bkey);
    d.brank = (uint2*)(A + L.brank);
    d.hlist = (uint32_t*)(A + L.hlist);
    d.counts = (unsigned long long*)(A + L.counts);
    d.digest = (unsigned long long*)(A + L.digest);
    {
        uint32_t* c = (uint32_t*)(A + L.simc);
        const size_t n = s->n_sims;
        d.sc.live = c;
        d.sc.dead[0] = c + n;
        d.sc.dead[1] = c + 2 * n;
        d.sc.born[0] = c + 3 * n;
        d.sc.born[1] = c + 4 * n;
        d.sc.next_id[0] = c + 5 * n;
        d.sc.next_id[1] = c + 6 * n;
    }
    d.head = (uint32_t*)(A + L.head);
    d.nxt = (uint32_t*)(A + L.nxt);
    d.glob = (uint32_t*)(A + L.glob);
    d.capacity = L.capacity;
    d.slots = L.slots;
    d.n_sims = s->n_sims;
    d.clist = (uint32_t*)(A + L.clist);
    d.ccount = (uint32_t*)(A + L.ccount);
    d.clist_cap = L.clist_cap;
}

// The neighbour search's mode (results do not depend on it): per chunk of
// sorted agents, or over the claimer list (single simulations only).  The
// list pays one atomic per wave that holds claimers when it is built, and
// deals the claimers evenly over the search's whole grid with at least 16
// lanes each, so `auto` takes it when claimers are under 1/64 of the
// initial agents (few claimers, often in crowded cells) or few enough to
// get 16 lanes each in one pass of the grid (small simulations, whose
// chunks are too few to fill the GPU).
void set_list_mode(mabm_sim* s)
{
    Dev& d = s->dev;
    bool list = false;
    if (s->n_sims == 1 && s->propose_mode != kModeChunks) {
        if (s->propose_mode == kModeList) {
            list = true;
        } else {
            const Tables& T = s->tabs[0];
            uint64_t claimers = 0, all = 0;
            for (int k = 0; k < T.ns; ++k) {
                const uint32_t c = T.init_end[k] - (k ? T.init_end[k - 1] : 0u);
                all += c;
                if (T.claimer[k]) claimers += c;
            }
            const uint64_t one_pass = (uint64_t)kListBlocks * 256u / 16u;
            list = claimers > 0 && (claimers * 64 < all || claimers <= one_pass);
        }
    }
    d.list_mode = list ? 1u : 0u;
    d.list_blocks = kListBlocks;
}

// first step / query / import: tables, hash geometry, upload, placement
mabm_status finalize(mabm_sim* s, bool place)
{
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    if (s->finalized) return MABM_OK;
    mabm_status st = build_tables(s);
    if (st != MABM_OK) return st;
    Dev& d = s->dev;
    const Tables& last = s->tabs.back();
    d.ncells = last.cell_base + (1u << (3 * last.morton_bits));
    // the fewest passes per scan tile that keep the tiles within the
    // arena's tile sums (the grid may be coarser than the one the arena
    // was sized for; fewer, longer tiles would put more of move's tile-sum
    // atomics on each counter)
    auto tiles = [&](uint32_t sh) {
        return ((size_t)d.ncells + ((size_t)kScanTile << sh) - 1) >> (kScanTileLog + sh);
    };
    d.tile_shift = 0;
    while (tiles(d.tile_shift) > s->lay.ntiles) ++d.tile_shift;
    d.ntiles = (uint32_t)tiles(d.tile_shift);
    // agents placed: every simulation's initial counts, one after another
    std::vector<uint32_t> n_init(s->n_sims);
    uint32_t total = 0;
    for (uint32_t k = 0; k < s->n_sims; ++k) {
        n_init[k] = place ? s->tabs[k].init_end[s->tabs[k].ns - 1] : 0;
        total += n_init[k];
    }
    d.n_init = total;
    HIP_OK(s, hipMemcpyAsync((void*)d.tab, s->tabs.data(), sizeof(Tables) * s->n_sims,
                             hipMemcpyHostToDevice, s->stream));
    Ctl c{};
    c.s[0] = StepState{0u, d.n_init, d.n_init, 0u};
    HIP_OK(s, hipMemcpyAsync(d.ctl, &c, sizeof c, hipMemcpyHostToDevice, s->stream));
    // per simulation: live agents and next ids from the placement, no
    // removals or children yet
    const size_t n = s->n_sims;
    s->host_simc.assign(kSimWords * n, 0u);
    for (size_t k = 0; k < n; ++k) {
        s->host_simc[k] = n_init[k];          // live
        s->host_simc[5 * n + k] = n_init[k];  // next_id[0]
    }
    HIP_OK(s, hipMemcpyAsync(d.sc.live, s->host_simc.data(), 4 * s->host_simc.size(),
                             hipMemcpyHostToDevice, s->stream));
    d.birth_blocks = has_births(s) ? kBirthSortBlocks : 0u;
    d.span = has_births(s) ? d.slots : d.capacity;
    // cell counts and both parities' tile sums start at zero
    HIP_OK(s, hipMemsetAsync(d.cell_count, 0, ((size_t)d.ntiles << (kScanTileLog + d.tile_shift)) * 4,
                             s->stream));
    HIP_OK(s, hipMemsetAsync(d.tile_acc, 0, (size_t)2 * d.ntiles * kTileStride * 4, s->stream));
    // claim slots are all-ones between steps (each step resets those it used)
    HIP_OK(s, hipMemsetAsync(d.slot, 0xFF, (size_t)d.slots * 8, s->stream));
    // the claimer list starts empty (each step's finish empties it again)
    HIP_OK(s, hipMemsetAsync(d.ccount, 0, (size_t)kListRegions * kListStride * 4, s->stream));
    set_list_mode(s);
    launch_fill_records(d, s->stream);
    if (place)
        for (uint32_t k = 0; k < s->n_sims; ++k) {
            Dev dk = d;  // the placement of simulation k with its own tables
            dk.tab = d.tab + k;
            dk.n_init = n_init[k];
            launch_init(dk, s->stream);
        }
    HIP_OK(s, hipGetLastError());
    HIP_OK(s, hipStreamSynchronize(s->stream));
    s->parity = 0;
    s->buf = 0;
    s->finalized = true;
    set_schedule(s);
    return MABM_OK;
}

// Synchronises the stream and reads the control block and the
// per-simulation counters; reports the sticky device errors, and checks the
// last step's end against each simulation's capacity (the device checks
// every earlier step's end at the start of the next one).
mabm_status sync_ctl(mabm_sim* s, Ctl* out)
{
    const size_t n = s->n_sims;
    s->host_simc.resize(kSimWords * n);
    HIP_OK(s, hipMemcpyAsync(out, s->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
    HIP_OK(s, hipMemcpyAsync(s->host_simc.data(), s->dev.sc.live, 4 * s->host_simc.size(),
                             hipMemcpyDeviceToHost, s->stream));
    HIP_OK(s, hipStreamSynchronize(s->stream));
    if (out->err) {
        s->failed = true;
        if (out->err & kErrPlacement) return fail(s, MABM_E_DEVICE, "initial placement failed after 64 attempts");
        if (out->err & kErrCapacity)
            return fail(s, MABM_E_CAPACITY, "live agents exceeded the capacity at the end of a step");
        return fail(s, MABM_E_CAPACITY,
                    "agent slots exhausted: one step's pair rules removed more agents than the "
                    "slot headroom (a quarter of the capacity) while the live agents were near it");
    }
    // the last step (parity s->parity ^ 1): live at its start, less its
    // removals, plus its children
    const int q = s->parity ^ 1;
    const uint32_t* c = s->host_simc.data();
    for (size_t k = 0; k < n; ++k) {
        const uint64_t live = (uint64_t)c[k] - c[(1 + q) * n + k] + c[(3 + q) * n + k];
        if (live > s->cfgs[k].capacity) {
            s->failed = true;
            return fail(s, MABM_E_CAPACITY,
                        "live agents exceeded the capacity at the end of a step (simulation " +
                            std::to_string(k) + ")");
        }
    }
    return MABM_OK;
}

mabm_status live_counts(mabm_sim* s, std::vector<unsigned long long>& out, Ctl* ctl)
{
    launch_counts(state_dev(s), s->parity, s->stream);
    HIP_OK(s, hipGetLastError());
    out.assign((size_t)kMaxSpecies * s->n_sims, 0ull);
    HIP_OK(s, hipMemcpyAsync(out.data(), s->dev.counts, out.size() * 8, hipMemcpyDeviceToHost,
                             s->stream));
    return sync_ctl(s, ctl);
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

}  // extern "C"

namespace {

// a batch's configurations must agree on everything but seed, volume size,
// capacity and cell size
bool batch_ok(const mabm_config* cs, uint32_t n, std::string& why)
{
    if (!cs || n == 0 || n > kMaxSims) {
        why = "a batch holds 1 to 65535 simulations";
        return false;
    }
    for (uint32_t k = 0; k < n; ++k) {
        if (!config_ok(&cs[k], why)) return false;
        if (cs[k].geometry != cs[0].geometry || cs[k].dt_s != cs[0].dt_s ||
            cs[k].flags != cs[0].flags) {
            why = "batch configurations differ in geometry, dt_s or flags";
            return false;
        }
    }
    if (total_capacity(cs, n) > (1ull << 30)) {
        why = "summed capacity of the batch above 2^30";
        return false;
    }
    uint64_t cells = 0;
    for (uint32_t k = 0; k < n; ++k) cells += (uint64_t)1 << (3 * morton_bits(grid_from_config(cs[k])));
    if (cells > kMaxCells) {
        why = "cell grids above 2^31 cells together (a larger cell_um gives fewer)";
        return false;
    }
    return true;
}

mabm_status create_impl(const mabm_config* cs, uint32_t n, void* device_arena, size_t arena_bytes,
                        void* hip_stream, mabm_sim** out)
{
    if (!out) return MABM_E_INVALID;
    *out = nullptr;
    std::string why;
    if (!batch_ok(cs, n, why)) {
        g_create_error = why;
        return MABM_E_INVALID;
    }
    Layout L = make_layout(cs, n);
    if (!device_arena || arena_bytes < L.total) {
        g_create_error = "arena smaller than mabm_arena_bytes()";
        return MABM_E_NOMEM;
    }
    if ((uintptr_t)device_arena % 256 != 0) {
        g_create_error = "arena must be 256-byte aligned";
        return MABM_E_INVALID;
    }
    mabm_sim* s = new (std::nothrow) mabm_sim();
    if (!s) return MABM_E_NOMEM;
    s->cfg = cs[0];
    s->cfgs.assign(cs, cs + n);
    s->n_sims = n;
    s->stream = (hipStream_t)hip_stream;
    s->arena = (uint8_t*)device_arena;
    s->arena_bytes = arena_bytes;
    s->lay = L;
    fill_dev(s);
    *out = s;
    return MABM_OK;
}

// The static arena of mabm_create_sim_static: device memory that needs no
// allocation call, for callers that cannot allocate.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// the array's name is no device address: the address on a device is taken
// once, with that device current, by hipGetSymbolAddress, and only that
// address is ever handed to kernels or copies.
constexpr size_t kStaticArenaBytes = size_t(64) << 20;
constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) uint8_t scratch[kStaticArenaBytes];

std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};
bool g_static_busy[kMaxStaticDevices] = {};

}  // namespace

extern "C" {

size_t mabm_arena_bytes(const mabm_config* cfg, uint32_t n_species, uint32_t n_rules)
{
    return mabm_batch_arena_bytes(cfg, 1, n_species, n_rules);
}

size_t mabm_batch_arena_bytes(const mabm_config* cfgs, uint32_t n_sims, uint32_t n_species,
                              uint32_t n_rules)
{
    std::string why;
    if (!batch_ok(cfgs, n_sims, why) || n_species > MABM_MAX_SPECIES || n_rules > MABM_MAX_RULES)
        return 0;
    return make_layout(cfgs, n_sims).total;
}

mabm_status mabm_create_sim(const mabm_config* cfg, void* device_arena, size_t arena_bytes,
                            void* hip_stream, mabm_sim** out)
{
    return create_impl(cfg, 1, device_arena, arena_bytes, hip_stream, out);
}

mabm_status mabm_create_batch(const mabm_config* cfgs, uint32_t n_sims, void* device_arena,
                              size_t arena_bytes, void* hip_stream, mabm_sim** out)
{
    return create_impl(cfgs, n_sims, device_arena, arena_bytes, hip_stream, out);
}

mabm_status mabm_create_sim_static(const mabm_config* cfg, void* hip_stream, mabm_sim** out)
{
    if (!out) return MABM_E_INVALID;
    *out = nullptr;
    std::string why;
    if (!batch_ok(cfg, 1, why)) {
        g_create_error = why;
        return MABM_E_INVALID;
    }
    const size_t need = make_layout(cfg, 1).total;
    if (need > kStaticArenaBytes) {
        g_create_error = "the configuration needs " + std::to_string(need) +
                         " device bytes; the static arena holds " +
                         std::to_string(kStaticArenaBytes) + " (use mabm_create_sim with an arena)";
        return MABM_E_NOMEM;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return MABM_E_DEVICE;
    }
    if (dev < 0 || dev >= kMaxStaticDevices) {
        g_create_error = "device index beyond the static arenas";
        return MABM_E_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev]) {
        g_create_error = "the static arena of this device holds a simulation already";
        return MABM_E_STATE;
    }
    if (!g_static_ptr[dev]) {
        // once per device, with the device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_create_error = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
            return MABM_E_DEVICE;
        }
        g_static_ptr[dev] = p;
    }
    // no graph is ever instantiated for it: steps are direct launches
    mabm_config c = *cfg;
    c.flags |= MABM_FLAG_NO_GRAPH;
    const mabm_status st = create_impl(&c, 1, g_static_ptr[dev], kStaticArenaBytes, hip_stream, out);
    if (st != MABM_OK) return st;
    (*out)->static_device = dev;
    g_static_busy[dev] = true;
    return MABM_OK;
}

mabm_status mabm_add_species(mabm_sim* s, const char* name, float D, uint32_t count, int32_t comp,
                             int32_t* out_id)
{
    if (!s) return MABM_E_INVALID;
    if (s->finalized || s->failed) return fail(s, MABM_E_STATE, "add_species after the model was finalized");
    if ((int)s->species.size() >= kMaxSpecies) return fail(s, MABM_E_INVALID, "too many species");
    const int ncomp = s->cfg.geometry == MABM_NESTED_SPHERES ? 2 : 1;
    if (!(D >= 0.0f) || !std::isfinite(D)) return fail(s, MABM_E_INVALID, "diffusion must be finite and >= 0");
    if (comp < 0 || comp >= ncomp) return fail(s, MABM_E_INVALID, "compartment does not exist in this geometry");
    s->species.push_back({name ? name : "", D, count, comp});
    s->sim_counts.emplace_back(s->n_sims, count);
    if (out_id) *out_id = (int32_t)s->species.size() - 1;
    return MABM_OK;
}

mabm_status mabm_set_initial_counts(mabm_sim* s, int32_t species_id, const uint32_t* counts)
{
    if (!s || !counts) return MABM_E_INVALID;
    if (s->finalized || s->failed) return fail(s, MABM_E_STATE, "initial counts after the model was finalized");
    if (species_id < 0 || species_id >= (int32_t)s->species.size())
        return fail(s, MABM_E_INVALID, "unknown species");
    s->sim_counts[species_id].assign(counts, counts + s->n_sims);
    return MABM_OK;
}

mabm_status mabm_add_rule(mabm_sim* s, const mabm_rule* r, int32_t* out_id)
{
    if (!s || !r) return MABM_E_INVALID;
    if (s->finalized || s->failed) return fail(s, MABM_E_STATE, "add_rule after the model was finalized");
    if ((int)s->rules.size() >= kMaxRules) return fail(s, MABM_E_INVALID, "too many rules");
    const int ns = (int)s->species.size();
    const int ncomp = s->cfg.geometry == MABM_NESTED_SPHERES ? 2 : 1;
    auto is_sp = [&](int v) { return v >= 0 && v < ns; };
    auto is_prod = [&](int v) { return v == -1 || is_sp(v); };
    if (!(r->prob_per_step >= 0.0 && r->prob_per_step <= 1.0))
        return fail(s, MABM_E_INVALID, "probability outside [0, 1]");
    if (!is_sp(r->reactant[0]) || !is_prod(r->product[0]) || !is_prod(r->product[1]))
        return fail(s, MABM_E_INVALID, "rule names an unknown species");
    if (r->kind == MABM_BIMOL) {
        if (!is_sp(r->reactant[1])) return fail(s, MABM_E_INVALID, "rule names an unknown species");
        if (r->placement != MABM_KEEP) return fail(s, MABM_E_INVALID, "bimolecular rules use KEEP");
        if (!(r->radius_um > 0.0f) || !std::isfinite(r->radius_um))
            return fail(s, MABM_E_INVALID, "contact radius must be > 0");
        for (const mabm_rule& o : s->rules)
            if (o.kind == MABM_BIMOL &&
                ((o.reactant[0] == r->reactant[0] && o.reactant[1] == r->reactant[1]) ||
                 (o.reactant[0] == r->reactant[1] && o.reactant[1] == r->reactant[0])))
                return fail(s, MABM_E_INVALID, "second bimolecular rule for one species pair");
    } else if (r->kind == MABM_UNIMOL) {
        if (r->reactant[1] != -1) return fail(s, MABM_E_INVALID, "unimolecular rule with two reactants");
        if (r->from_comp < -1 || r->from_comp >= ncomp) return fail(s, MABM_E_INVALID, "bad compartment");
        switch (r->placement) {
        case MABM_KEEP:
            if (r->product[1] != -1) return fail(s, MABM_E_INVALID, "KEEP has one product");
            break;
        case MABM_SPLIT:
        case MABM_EMIT:
            if (r->placement == MABM_SPLIT && r->product[0] < 0)
                return fail(s, MABM_E_INVALID, "SPLIT needs two products");
            if (r->product[1] < 0) return fail(s, MABM_E_INVALID, "missing emitted product");
            if (!(r->release_radius_um >= 0.0f) || !std::isfinite(r->release_radius_um))
                return fail(s, MABM_E_INVALID, "bad release radius");
            break;
        case MABM_TRANSLOCATE: {
            if (s->cfg.geometry != MABM_NESTED_SPHERES)
                return fail(s, MABM_E_INVALID, "translocation needs nested compartments");
            if (r->from_comp < 0 || r->to_comp < 0 || r->to_comp >= ncomp || r->to_comp == r->from_comp)
                return fail(s, MABM_E_INVALID, "bad translocation compartments");
            if (r->product[1] != -1) return fail(s, MABM_E_INVALID, "TRANSLOCATE has one product");
            for (const mabm_config& c : s->cfgs) {
                const double rt = r->to_comp == 0
                                      ? (double)c.inner_radius_um - (double)r->release_radius_um
                                      : (double)c.inner_radius_um + (double)r->release_radius_um;
                if (!(r->release_radius_um >= 1e-3f) || !(rt > 0.0) || !(rt < (double)c.outer_radius_um))
                    return fail(s, MABM_E_INVALID, "bad translocation offset");
            }
            break;
        }
        default:
            return fail(s, MABM_E_INVALID, "bad placement");
        }
    } else {
        return fail(s, MABM_E_INVALID, "bad rule kind");
    }
    s->rules.push_back(*r);
    if (out_id) *out_id = (int32_t)s->rules.size() - 1;
    return MABM_OK;
}

mabm_status mabm_grid(mabm_sim* s, uint32_t* g, float* h)
{
    if (!s) return MABM_E_INVALID;
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (g) *g = s->G;
    if (h) *h = s->h;
    return MABM_OK;
}

}  // extern "C"

namespace {

// one step of parity p on the agents in buffer `buf`: move, scan and
// scatter into the other buffer (bin; a step that keeps the cell lists has
// neither), then [propose, finish]
void enqueue_step(mabm_sim* s, int p, int buf, bool bin, uint32_t moved)
{
    Dev d = s->dev;
    d.a[p] = s->dev.a[buf];
    d.a[p ^ 1] = s->dev.a[bin ? buf ^ 1 : buf];
    const int rec = (s->cfg.flags & MABM_FLAG_RECORD) ? 1 : 0;
    hipStream_t q = s->stream;
    timed(s, kKMove, [&](const KEvents& e) { launch_move(d, p, rec, bin ? 1 : 0, moved, q, e); });
    if (bin) {
        timed(s, kKScan, [&](const KEvents& e) { launch_scan(d, p, q, e); });
        timed(s, kKScatter, [&](const KEvents& e) { launch_scatter(d, p, rec, q, e); });
    }
    // (only models with pair rules keep cell lists)
    if (s->has_bimol) {
        const int b = bin ? 1 : 0;
        timed(s, kKPropose, [&](const KEvents& e) { launch_propose(d, p, b, moved, q, e); });
        timed(s, kKFinish, [&](const KEvents& e) { launch_finish(d, p, rec, b, q, e); });
    }
}

// Capture `steps` consecutive steps from the current schedule state as one graph on
// the caller's stream (kernel nodes only: the step has no memset or copy).
// Long runs replay the multi-step graph, so the host issues one launch per
// graph_steps steps; that matters for small simulations, whose steps take
// about as long to enqueue as to run.  The multi-step graph spans at least
// 16 steps and a whole number of pairs of binning cycles, so it ends in the
// state it starts from (parity, buffer, steps since the binning) and one
// capture serves the whole run.
constexpr uint32_t kGraphSteps = 16;

uint32_t graph_steps(const mabm_sim* s)
{
    const uint32_t cycle = 2 * s->bin_every;
    return (kGraphSteps + cycle - 1) / cycle * cycle;
}

// Advances the schedule state (parity, buffer, steps kept) by one step;
// returns whether that step bins.
bool advance(mabm_sim* s)
{
    const bool bin = bins(s, s->kept);
    s->parity ^= 1;
    if (bin) {
        s->buf ^= 1;
        s->kept = 0;
    } else {
        ++s->kept;
    }
    return bin;
}

// Enqueues `steps` steps from the current schedule state and advances it.
void enqueue_steps(mabm_sim* s, uint32_t steps)
{
    for (uint32_t k = 0; k < steps; ++k) {
        const int p = s->parity, b = s->buf;
        const uint32_t moved = s->kept + 1;  // moves since the binning, if this step keeps it
        const bool bin = advance(s);
        enqueue_step(s, p, b, bin, bin ? 0u : moved);
    }
}

mabm_status capture(mabm_sim* s, uint32_t steps, hipGraphExec_t* out)
{
    hipGraph_t g = nullptr;
    // the schedule state is restored: the graph is launched after capture
    const int parity = s->parity, buf = s->buf;
    const uint32_t kept = s->kept;
    HIP_OK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    enqueue_steps(s, steps);
    s->parity = parity;
    s->buf = buf;
    s->kept = kept;
    HIP_OK(s, hipStreamEndCapture(s->stream, &g));
    const hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
    return MABM_OK;
}

}  // namespace

extern "C" {

mabm_status mabm_step(mabm_sim* s, uint32_t n_steps)
{
    if (!s) return MABM_E_INVALID;
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    // graphs need a capturable (non-null) stream; per-kernel timing records
    // events between the kernels, so it launches them directly
    const bool graphs = s->stream != nullptr && !s->prof && !(s->cfg.flags & MABM_FLAG_NO_GRAPH);
    uint32_t k = 0;
    while (k < n_steps) {
        uint32_t m = 1;
        // steps until the next counts-ring entry (a graph never spans one)
        const uint64_t until_rec =
            s->ring_every ? s->ring_every - s->steps_done % s->ring_every : ~0ull;
        if (graphs) {
            const uint32_t L = graph_steps(s);
            const uint32_t kind = (n_steps - k >= L && until_rec >= L) ? 1 : 0;
            m = kind ? L : 1u;
            const uint32_t key = kind | uint32_t(s->parity) << 1 | uint32_t(s->buf) << 2 | s->kept << 3;
            hipGraphExec_t& g = s->graphs[key];
            if (!g) {
                st = capture(s, m, &g);
                if (st != MABM_OK) {
                    s->graphs.erase(key);
                    return st;
                }
            }
            HIP_OK(s, hipGraphLaunch(g, s->stream));
            for (uint32_t j = 0; j < m; ++j) advance(s);  // the state the graph leaves
        } else {
            enqueue_steps(s, 1);
        }
        s->steps_done += m;
        k += m;
        if (s->ring_every && s->steps_done % s->ring_every == 0) {
            unsigned long long* e =
                s->ring + (s->ring_recorded % s->ring_entries) * ring_words(s);
            launch_counts(state_dev(s), s->parity, s->stream, e + 1, e);
            ++s->ring_recorded;
        }
    }
    HIP_OK(s, hipGetLastError());
    return MABM_OK;
}

mabm_status mabm_counts(mabm_sim* s, uint64_t* out, uint32_t n_species, uint64_t* out_step)
{
    if (!s) return MABM_E_INVALID;
    if (!out && n_species) return fail(s, MABM_E_INVALID, "null counts array");
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    std::vector<unsigned long long> c;
    Ctl ctl{};
    st = live_counts(s, c, &ctl);
    if (st != MABM_OK) return st;
    for (uint32_t k = 0; k < n_species; ++k) {
        uint64_t v = 0;
        if (k < (uint32_t)kMaxSpecies)
            for (uint32_t m = 0; m < s->n_sims; ++m) v += c[(size_t)m * kMaxSpecies + k];
        out[k] = v;
    }
    if (out_step) *out_step = ctl.s[s->parity].t;
    return MABM_OK;
}

mabm_status mabm_size(mabm_sim* s, uint32_t* n_live, uint32_t* next_id)
{
    if (!s) return MABM_E_INVALID;
    if (is_batch(s, "mabm_size")) return MABM_E_STATE;
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    std::vector<unsigned long long> c;
    Ctl ctl{};
    st = live_counts(s, c, &ctl);
    if (st != MABM_OK) return st;
    if (n_live) *n_live = (uint32_t)std::accumulate(c.begin(), c.end(), 0ull);
    if (next_id) *next_id = ctl.s[s->parity].next_id;
    return MABM_OK;
}

}  // extern "C"

namespace {

// live agents of simulation `sim` (a single simulation: 0), sorted by id
mabm_status export_impl(mabm_sim* s, uint32_t sim, uint32_t capacity, uint32_t* id,
                        uint8_t* species, float* x, float* y, float* z, uint32_t* key,
                        int32_t* event, uint32_t* partner)
{
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    Ctl ctl{};
    st = sync_ctl(s, &ctl);
    if (st != MABM_OK) return st;
    // the device gathers the simulation's live agents (wherever births and
    // holes have put them) into arrays that are free between steps
    const bool rec = (s->cfg.flags & MABM_FLAG_RECORD) != 0;
    Dev d = state_dev(s);
    HIP_OK(s, hipMemsetAsync(&d.ctl->export_n, 0, 4, s->stream));
    launch_export(d, s->parity, sim, rec ? 1 : 0, s->stream);
    HIP_OK(s, hipGetLastError());
    uint32_t n = 0;
    HIP_OK(s, hipMemcpyAsync(&n, &d.ctl->export_n, 4, hipMemcpyDeviceToHost, s->stream));
    HIP_OK(s, hipStreamSynchronize(s->stream));
    if (n > d.capacity) return fail(s, MABM_E_CAPACITY, "more live agents than the capacity");
    if (n > capacity) return fail(s, MABM_E_INVALID, "export buffer smaller than the live agents");
    std::vector<Birth> hb(n);
    std::vector<unsigned long long> hk(rec ? n : 0);
    std::vector<uint8_t> he(rec ? n : 0);
    if (n) {
        HIP_OK(s, hipMemcpyAsync(hb.data(), d.births, (size_t)n * sizeof(Birth), hipMemcpyDeviceToHost,
                                 s->stream));
        if (rec) {
            HIP_OK(s, hipMemcpyAsync(hk.data(), d.bkey, (size_t)n * 8, hipMemcpyDeviceToHost, s->stream));
            HIP_OK(s, hipMemcpyAsync(he.data(), d.event, n, hipMemcpyDeviceToHost, s->stream));
        }
        HIP_OK(s, hipStreamSynchronize(s->stream));
    }
    std::vector<uint32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0u);
    std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return hb[a].parent < hb[b].parent; });
    for (size_t k = 0; k < n; ++k) {
        const Birth& g = hb[idx[k]];
        if (id) id[k] = g.parent;
        if (species) species[k] = (uint8_t)(g.sp & 0xFFu);
        if (x) x[k] = g.x;
        if (y) y[k] = g.y;
        if (z) z[k] = g.z;
        if (key) key[k] = rec ? (uint32_t)(hk[idx[k]] >> 32) : MABM_NONE;
        if (event) event[k] = (rec && he[idx[k]] != kNoEvent) ? (int32_t)he[idx[k]] : -1;
        if (partner) partner[k] = rec ? (uint32_t)hk[idx[k]] : MABM_NONE;
    }
    return MABM_OK;
}

}  // namespace

extern "C" {

mabm_status mabm_export(mabm_sim* s, uint32_t capacity, uint32_t* id, uint8_t* species, float* x,
                        float* y, float* z, uint32_t* key, int32_t* event, uint32_t* partner)
{
    if (!s) return MABM_E_INVALID;
    if (is_batch(s, "mabm_export")) return MABM_E_STATE;
    return export_impl(s, 0, capacity, id, species, x, y, z, key, event, partner);
}

mabm_status mabm_import(mabm_sim* s, uint32_t n, const uint32_t* id, const uint8_t* sp,
                        const float* x, const float* y, const float* z, uint32_t next_id, uint32_t t)
{
    if (!s) return MABM_E_INVALID;
    if (is_batch(s, "mabm_import")) return MABM_E_STATE;
    if (s->finalized) return fail(s, MABM_E_STATE, "import after the model was finalized");
    if (n > s->cfg.capacity) return fail(s, MABM_E_CAPACITY, "import exceeds the capacity");
    if (n && (!id || !sp || !x || !y || !z)) return fail(s, MABM_E_INVALID, "null import array");
    const mabm_config& c = s->cfg;
    const float Rout2 = (float)((double)c.outer_radius_um * (double)c.outer_radius_um);
    for (uint32_t i = 0; i < n; ++i) {
        if (sp[i] >= s->species.size()) return fail(s, MABM_E_INVALID, "unknown species in import");
        if (id[i] >= next_id) return fail(s, MABM_E_INVALID, "id not below next_id");
        if (c.geometry == MABM_PERIODIC_BOX) {
            if (!(x[i] >= 0.0f && x[i] < c.box_um && y[i] >= 0.0f && y[i] < c.box_um && z[i] >= 0.0f &&
                  z[i] < c.box_um))
                return fail(s, MABM_E_INVALID, "imported position outside the box");
        } else if (!(x[i] * x[i] + y[i] * y[i] + z[i] * z[i] <= Rout2)) {
            return fail(s, MABM_E_INVALID, "imported position outside the volume");
        }
    }
    {
        // ids key every random draw, so each may appear once
        std::vector<uint32_t> ids(id, id + n);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
            return fail(s, MABM_E_INVALID, "duplicate id in import");
    }
    mabm_status st = finalize(s, false);
    if (st != MABM_OK) return st;
    const Agents& A = s->dev.a[0];
    std::vector<uint4> hr(n);
    for (uint32_t i = 0; i < n; ++i) {
        std::memcpy(&hr[i].x, &x[i], 4);
        std::memcpy(&hr[i].y, &y[i], 4);
        std::memcpy(&hr[i].z, &z[i], 4);
        hr[i].w = sp[i];
    }
    if (n) {
        HIP_OK(s, hipMemcpyAsync(A.rec, hr.data(), (size_t)n * 16, hipMemcpyHostToDevice, s->stream));
        HIP_OK(s, hipMemcpyAsync(A.id, id, n * 4, hipMemcpyHostToDevice, s->stream));
    }
    Ctl ctl{};
    ctl.s[0] = StepState{t, n, next_id, 0u};
    HIP_OK(s, hipMemcpyAsync(s->dev.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s->stream));
    // one simulation: n live agents, ids from next_id
    s->host_simc.assign(kSimWords, 0u);
    s->host_simc[0] = n;
    s->host_simc[5] = next_id;
    HIP_OK(s, hipMemcpyAsync(s->dev.sc.live, s->host_simc.data(), 4 * kSimWords, hipMemcpyHostToDevice,
                             s->stream));
    HIP_OK(s, hipStreamSynchronize(s->stream));
    s->parity = 0;
    s->buf = 0;
    s->kept = s->bin_every - 1;  // imported agents are not binned
    return MABM_OK;
}

mabm_status mabm_profile(mabm_sim* s, int32_t enable)
{
    if (!s) return MABM_E_INVALID;
    if (enable && s->pool.empty()) {
        s->pool.resize(8192);
        s->pending_kernel.resize(8192);
        for (EventPair& p : s->pool) {
            HIP_OK(s, hipEventCreate(&p.a));
            HIP_OK(s, hipEventCreate(&p.b));
        }
    }
    if (!enable) harvest(s);
    s->prof = enable != 0;
    for (int k = 0; k < kNumKernels; ++k) {
        s->launches[k] = 0;
        s->total_ms[k] = 0.0;
    }
    s->pending = 0;
    return MABM_OK;
}

mabm_status mabm_profile_read(mabm_sim* s, const char** names, uint64_t* launches, double* total_ms)
{
    if (!s) return MABM_E_INVALID;
    harvest(s);
    for (int k = 0; k < kNumKernels; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (launches) launches[k] = s->launches[k];
        if (total_ms) total_ms[k] = s->total_ms[k];
    }
    return MABM_OK;
}

mabm_status mabm_batch_counts(mabm_sim* s, uint64_t* out, uint32_t n_species, uint64_t* out_step)
{
    if (!s || !out) return MABM_E_INVALID;
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    std::vector<unsigned long long> c;
    Ctl ctl{};
    st = live_counts(s, c, &ctl);
    if (st != MABM_OK) return st;
    for (uint32_t m = 0; m < s->n_sims; ++m)
        for (uint32_t k = 0; k < n_species; ++k)
            out[(size_t)m * n_species + k] =
                k < (uint32_t)kMaxSpecies ? c[(size_t)m * kMaxSpecies + k] : 0;
    if (out_step) *out_step = ctl.s[s->parity].t;
    return MABM_OK;
}

mabm_status mabm_batch_size(mabm_sim* s, uint32_t sim, uint32_t* n_live, uint32_t* next_id)
{
    if (!s) return MABM_E_INVALID;
    if (sim >= s->n_sims) return fail(s, MABM_E_INVALID, "simulation index out of range");
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    std::vector<unsigned long long> c;
    Ctl ctl{};
    st = live_counts(s, c, &ctl);
    if (st != MABM_OK) return st;
    if (n_live)
        *n_live = (uint32_t)std::accumulate(c.begin() + (size_t)sim * kMaxSpecies,
                                            c.begin() + (size_t)(sim + 1) * kMaxSpecies, 0ull);
    if (next_id) {
        // sync_ctl (through live_counts) read the per-simulation counters
        *next_id = s->host_simc[(5 + s->parity) * s->n_sims + sim];
    }
    return MABM_OK;
}

mabm_status mabm_batch_export(mabm_sim* s, uint32_t sim, uint32_t capacity, uint32_t* id,
                              uint8_t* species, float* x, float* y, float* z, uint32_t* key,
                              int32_t* event, uint32_t* partner)
{
    if (!s) return MABM_E_INVALID;
    if (sim >= s->n_sims) return fail(s, MABM_E_INVALID, "simulation index out of range");
    return export_impl(s, sim, capacity, id, species, x, y, z, key, event, partner);
}

mabm_status mabm_batch_grid(mabm_sim* s, uint32_t sim, uint32_t* g, float* h)
{
    if (!s) return MABM_E_INVALID;
    if (sim >= s->n_sims) return fail(s, MABM_E_INVALID, "simulation index out of range");
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (g) *g = s->sim_G[sim];
    if (h) *h = s->sim_h[sim];
    return MABM_OK;
}

size_t mabm_ring_entry_bytes(const mabm_sim* s) { return s ? 8 * ring_words(s) : 0; }

mabm_status mabm_counts_ring(mabm_sim* s, void* device_ring, uint32_t entries, uint32_t every)
{
    if (!s) return MABM_E_INVALID;
    if (every && (!device_ring || entries == 0 || (uintptr_t)device_ring % 8 != 0))
        return fail(s, MABM_E_INVALID, "counts ring needs an 8-byte aligned buffer of >= 1 entry");
    // steps already enqueued may still write the old ring: it is released
    // only once they have run
    if (s->ring) HIP_OK(s, hipStreamSynchronize(s->stream));
    s->ring = every ? (unsigned long long*)device_ring : nullptr;
    s->ring_entries = every ? entries : 0;
    s->ring_every = every;
    s->ring_recorded = 0;
    return MABM_OK;
}

mabm_status mabm_ring_read(mabm_sim* s, uint64_t* out, uint32_t max_entries, uint64_t* n_recorded)
{
    if (!s) return MABM_E_INVALID;
    if (n_recorded) *n_recorded = s->ring_recorded;
    if (!s->ring || !out || max_entries == 0) return MABM_OK;
    HIP_OK(s, hipStreamSynchronize(s->stream));
    const uint64_t held = std::min<uint64_t>(s->ring_recorded, s->ring_entries);
    const uint64_t n = std::min<uint64_t>(held, max_entries);
    const size_t w = ring_words(s);
    for (uint64_t k = 0; k < n; ++k) {  // the last n entries, oldest first
        const uint64_t idx = (s->ring_recorded - n + k) % s->ring_entries;
        HIP_OK(s, hipMemcpy(out + k * w, s->ring + idx * w, w * 8, hipMemcpyDeviceToHost));
    }
    return MABM_OK;
}

mabm_status mabm_set_param(mabm_sim* s, int32_t param, uint32_t value)
{
    if (!s) return MABM_E_INVALID;
    // captured steps hold the old launch shape and schedule
    HIP_OK(s, hipStreamSynchronize(s->stream));
    drop_graphs(s);
    switch (param) {
    case MABM_PARAM_PROPOSE_LANES: {
        // a power of two that covers the stencil with at most two cells per lane
        const bool ok = value == 0 || value == 4 || value == 8 || value == 16 || value == 32;
        if (!ok) return fail(s, MABM_E_INVALID, "lanes per claimer must be 0, 4, 8, 16 or 32");
        s->dev.prop_lanes = value;
        return MABM_OK;
    }
    case MABM_PARAM_PROPOSE_MIN_WORKGROUPS:
        if (value > (1u << 20)) return fail(s, MABM_E_INVALID, "at most 2^20 workgroups");
        s->dev.prop_min_blocks = value;
        return MABM_OK;
    case MABM_PARAM_PROPOSE_MODE:
        if (value > kModeList) return fail(s, MABM_E_INVALID, "search mode must be 0, 1 or 2");
        if (value == kModeList && s->n_sims > 1)
            return fail(s, MABM_E_INVALID, "the claimer-list search serves single simulations");
        s->propose_mode = value;
        if (s->finalized) set_list_mode(s);
        return MABM_OK;
    case MABM_PARAM_BIN_EVERY_MAX:
        if (value > kMaxBinEvery) return fail(s, MABM_E_INVALID, "at most 8 steps between binnings");
        s->bin_every_max = value;
        if (s->finalized) set_schedule(s);
        return MABM_OK;
    default:
        return fail(s, MABM_E_INVALID, "unknown parameter");
    }
}

mabm_status mabm_get_param(mabm_sim* s, int32_t param, uint32_t* value)
{
    if (!s || !value) return MABM_E_INVALID;
    switch (param) {
    case MABM_PARAM_PROPOSE_LANES: *value = s->dev.prop_lanes; return MABM_OK;
    case MABM_PARAM_PROPOSE_MIN_WORKGROUPS: *value = s->dev.prop_min_blocks; return MABM_OK;
    case MABM_PARAM_BIN_EVERY_MAX: *value = s->bin_every_max; return MABM_OK;
    case MABM_PARAM_PROPOSE_MODE: {
        // the mode in use (1 or 2), once the model is final
        mabm_status st = finalize(s, true);
        if (st != MABM_OK) return st;
        *value = s->dev.list_mode ? kModeList : kModeChunks;
        return MABM_OK;
    }
    case MABM_PARAM_BIN_EVERY: {
        mabm_status st = finalize(s, true);
        if (st != MABM_OK) return st;
        *value = s->bin_every;
        return MABM_OK;
    }
    default: return fail(s, MABM_E_INVALID, "unknown parameter");
    }
}

mabm_status mabm_digest(mabm_sim* s, uint64_t* out, uint32_t n)
{
    if (!s || !out) return MABM_E_INVALID;
    if (n != s->n_sims) return fail(s, MABM_E_INVALID, "digest array must have one entry per simulation");
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    if (s->failed) return fail(s, MABM_E_STATE, "simulation has failed: " + s->err);
    launch_digest(state_dev(s), s->parity, s->dev.digest, s->stream);
    HIP_OK(s, hipGetLastError());
    HIP_OK(s, hipMemcpyAsync(out, s->dev.digest, (size_t)8 * n, hipMemcpyDeviceToHost, s->stream));
    Ctl ctl{};
    return sync_ctl(s, &ctl);
}

mabm_status mabm_agent_updates(mabm_sim* s, uint64_t* out)
{
    if (!s || !out) return MABM_E_INVALID;
    mabm_status st = finalize(s, true);
    if (st != MABM_OK) return st;
    Ctl ctl{};
    st = sync_ctl(s, &ctl);
    if (st != MABM_OK) return st;
    *out = ctl.agent_updates;
    return MABM_OK;
}

mabm_status mabm_destroy_sim(mabm_sim* s)
{
    if (!s) return MABM_E_INVALID;
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (EventPair& p : s->pool) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    if (s->static_device >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[s->static_device] = false;
    }
    delete s;
    return MABM_OK;
}

const char* mabm_last_error(const mabm_sim* s)
{
    if (!s) return g_create_error.c_str();
    return s->err.c_str();
}

}  // extern "C"
