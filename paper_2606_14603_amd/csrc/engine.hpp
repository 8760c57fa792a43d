// engine.hpp -- internal layout shared by the kernels and the host engine of
// libmabm (device tables, control block, arena pointers, launch entry
// points).  Not part of the public ABI (include/mabm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mabm {

constexpr int kMaxSpecies = 64;
constexpr int kMaxRules = 255;
constexpr int kMaxUni = 8;        // unimolecular rules per (species, compartment)
constexpr uint8_t kDead = 0xFF;   // species byte of a consumed agent (hole)
constexpr uint8_t kNoEvent = 0xFF;
constexpr uint8_t kNoRule = 0xFF;  // no pair rule (rule indices run to kMaxRules - 1)
static_assert(kMaxRules <= 255, "rule indices fit a byte beside kNoRule");
// An agent is a 16-byte record {x, y, z, meta} (position bits, then
// species in bits 0-7, this step's flags in bits 8-15 and, in a batch, the
// index of the agent's simulation in bits 16-31) plus its id in a separate
// array.
constexpr uint32_t kMetaBusy = 1u << 8;     // had a unimolecular event this step
constexpr uint32_t kMetaClaimer = 1u << 9;  // non-busy agent of a claiming species
constexpr uint32_t kMetaListed = 1u << 10;  // a hole already in the hole list
constexpr uint32_t kMetaSimShift = 16;
constexpr uint32_t kMetaSimMask = 0xFFFF0000u;
constexpr uint32_t kMaxSims = 65535;
constexpr int kMetaSpeciesByte = 12;        // byte offset of the species in a record
constexpr uint32_t kNone = 0xFFFFFFFFu;
// Extra cell lists of a kept binning: agents placed since the binning
// (newborns, translocated agents, split parents) are chained per cell
// through `nxt`; kEnd ends a chain, kUnlinked marks a slot in no chain, and
// kGlobBit a chained slot placed again, which then sits in the global list
// every claimer reads.
constexpr uint32_t kEnd = 0x7FFFFFFFu;
constexpr uint32_t kUnlinked = 0x7FFFFFFEu;
constexpr uint32_t kGlobBit = 0x80000000u;

// Claimer list (the search mode for sparse claimers): the step's claimers,
// appended by the kernel that flags them (scatter in a binning step, move in
// a step that keeps the binning) into kListRegions regions, each with its
// own counter on its own 128-byte line (a workgroup appends to region
// blockIdx mod kListRegions, one atomic per wave); an entry is the
// claimer's slot, with kListWide set when it searches the 27-cell stencil.
constexpr uint32_t kListRegions = 64;
constexpr uint32_t kListStride = 32;  // words between region counters
constexpr uint32_t kListWide = 0x80000000u;
// Births of a step are ranked by (simulation, parent id): runs of kBirthRun
// records are sorted in LDS by kBirthSortBlocks workgroups, and each birth's
// rank is its rank in its own run plus its lower bound in every other run.
constexpr uint32_t kBirthRun = 256;
constexpr uint32_t kBirthRunLog = 8;
static_assert(kBirthRun == 1u << kBirthRunLog, "birth runs are a power of two");
constexpr uint32_t kBirthSortBlocks = 32;
constexpr uint32_t kTileStride = 1024;        // words between tile counters (4 KiB)
constexpr int kScanItems = 8;                 // cells per thread in the scan
constexpr int kScanThreads = 256;
constexpr int kScanTile = kScanItems * kScanThreads;  // cells per scan pass of a workgroup
constexpr int kScanTileLog = 11;
static_assert(kScanTile == 1 << kScanTileLog, "scan tile is a power of two");
// A scan tile (one workgroup of the scan, one counter of the per-tile sums)
// spans 2^tile_shift passes of kScanTile cells, the smallest power that
// keeps the number of tiles at most kMaxScanTiles.
constexpr uint32_t kMaxScanTiles = 1024;
// sorted agents per workgroup of the neighbour search; the claimer-flag
// array is padded to a whole number of these
constexpr uint32_t kClaimChunk = 1024;

// Philox counter "purpose" words (third counter word; 1 is unused: the
// event draw shares the MOVE block).
enum Purpose : uint32_t { kInit = 0, kMove = 2, kPair = 3, kPrio = 4, kBirth = 5 };

enum Geometry : int32_t { kBox = 0, kSphere = 1, kNested = 2 };
enum Placement : int32_t { kKeep = 0, kSplit = 1, kEmit = 2, kTranslocate = 3 };

// sticky device error bits: a simulation's live agents above its capacity
// at a step's end; an initial placement that failed; more slots needed than
// the arrays hold (the capacity plus the headroom for holes, see Dev::slots)
enum ErrBit : uint32_t { kErrCapacity = 1u, kErrPlacement = 2u, kErrSlots = 4u };

struct RuleDev {
    int32_t kind, placement, p0, p1, to;
    float r2;        // squared contact radius (BIMOL)
    float release;   // release-ball radius / translocation offset
    float release2;  // squared release radius
    float target_r;  // translocation landing radius
    uint32_t pad;
    uint64_t thr;    // Bernoulli threshold in [0, 2^32] (BIMOL)
};

// What move needs of a species in a compartment, in one 32-byte read: its
// step sigma, its first unimolecular rule and that rule's threshold
// (`always` when it is 2^32), and, as a claimer, its largest contact radius
// and its targets' largest move per step.
struct SpecHot {
    float sigma;
    uint32_t thr0;
    float rmax, dmax;
    uint8_t uni_n, rule0, claimer, always;
    uint32_t pad[3];
};
static_assert(sizeof(SpecHot) == 32, "one 32-byte read");

struct Tables {
    int32_t geometry, ncomp, ns, nr;
    float L, halfL, Rout, Rout2, Rin, Rin2;
    float lo, inv_h;
    uint32_t G, stencil8;  // cells per axis; 1 = 8-cell stencil (h >= 2 R_max)
    uint32_t morton_bits;  // cells are sorted by the Morton (Z-order) index of their
                           // coordinates over a 2^bits grid per axis
    uint32_t key0, key1;   // Philox key (seed low, high)
    uint32_t capacity;     // the simulation's most live agents at a step's end
    uint32_t pad1;
    // position of this simulation in a batch (all zero for a single one):
    // its index, its first cell in the batch's cell order, its first slot
    // at placement
    uint32_t sim, cell_base, slot_base, pad2;
    uint32_t init_end[kMaxSpecies];  // prefix sums of initial counts (placement)
    int32_t init_comp[kMaxSpecies];
    float sigma[kMaxSpecies];
    uint8_t claimer[kMaxSpecies];
    float claim_r2max[kMaxSpecies];  // largest squared contact radius of a claimer's rules
    float claim_rmax[kMaxSpecies];   // and that radius (um)
    // per claimer species: how far (um, along an axis) one step can move any
    // agent that is, or can later become, a target of its rules
    float claim_dmax[kMaxSpecies];
    uint8_t uni_n[kMaxSpecies][2];
    uint8_t uni_rule[kMaxSpecies][2][kMaxUni];
    uint64_t uni_thr[kMaxSpecies][2][kMaxUni];
    uint8_t rule_of[kMaxSpecies][kMaxSpecies];  // pair rule of (claimer, target), kNoRule: none
    RuleDev rule[kMaxRules];
    SpecHot hot[kMaxSpecies][2];  // [species][compartment], from the fields above
};

// Step scalars are double-buffered by parity p = t mod 2 (the buffer the
// step starts from): the kernels of a step read side p, and the step's last
// bookkeeping writes side p ^ 1 for the next step, so no kernel of a step
// ever sees the next step's values.
struct StepState {
    uint32_t t;        // step counter
    uint32_t n_slots;  // entries of the agent arrays (holes included)
    uint32_t next_id;  // (a single simulation; a batch keeps one per simulation)
    uint32_t h_used;   // entries of the hole list already refilled by births
};

struct Ctl {
    StepState s[2];
    uint32_t n_births[2];  // birth records appended by the step of parity p
    uint32_t n_prop[2];    // entries of the proposer list of the step of parity p
    uint32_t n_binned;     // agents binned by the last binning (births follow them)
    uint32_t h_n;          // entries of the hole list since the last binning
    uint32_t n_glob;       // entries of the global list of agents placed again
    uint32_t export_n;     // agents gathered by the last export
    uint32_t err;          // ErrBit, sticky
    uint32_t pad;
    unsigned long long agent_updates;  // sum of live agents at step starts
};

// Per-simulation counters, n_sims entries each, the step-indexed ones
// double-buffered by parity like the step scalars: live agents at the
// current step's start; agents removed and born by the step of parity p;
// the next id to assign at the start of the step of parity p.
struct SimCounters {
    uint32_t* live;
    uint32_t* dead[2];
    uint32_t* born[2];
    uint32_t* next_id[2];
};

struct Birth {
    uint32_t parent, sp;  // sp: species, and the simulation index in bits 16-31
    float x, y, z;
};

struct Agents {
    uint4* rec;
    uint32_t* id;
};

struct Dev {
    Ctl* ctl;
    const Tables* tab;
    Agents a[2];          // ping-pong agent arrays
    uint32_t* rank;       // per pre-sort slot: rank in its cell (kNone: not binned)
    uint8_t* event;       // per pre-sort slot: event rule (record mode)
    uint8_t* sclaim;      // per agent slot: 1 = claimer this step, 2 = one searching
                          // the 27-cell stencil while the others search 8
    uint32_t* cell_count;  // ncells rounded up to whole scan tiles
    uint32_t* cell_start;  // padded ncells + 1
    uint32_t* tile_acc;    // [2][ntiles * kTileStride]: cell-count sums per scan tile,
                           // accumulated by move, one set per parity
    unsigned long long* slot;
    uint32_t* prop;        // per sorted agent: proposed partner index
    uint4* plist;          // this step's proposals {claimer, target, their ids}
    uint32_t* rkey;        // record arrays, indexed like the current agents
    uint8_t* revent;
    uint32_t* rpartner;
    Birth* births;               // this step's birth records (births_cap)
    unsigned long long* bkey;    // birth runs sorted by (simulation << 32 | parent id)
    uint2* brank;                // per birth record: its rank in its run, and the
                                 // records of smaller simulations in the run
    uint32_t* hlist;             // slots of holes since the binning (kept steps refill them)
    unsigned long long* counts;  // [n_sims][kMaxSpecies]
    unsigned long long* digest;  // [n_sims], state digests (queries only)
    SimCounters sc;
    uint32_t* head;              // per cell: first agent of its extra chain (kEnd: none)
    uint32_t* nxt;               // per slot: next agent of its chain, kUnlinked, kGlobBit
    uint32_t* glob;              // agents placed twice since the binning
    uint32_t link;               // keep extra chains (kept binnings with placements)
    // capacity: live agents of all simulations together (the sum of their
    // capacities), which also bounds the births of a step; slots: entries of
    // the agent arrays, the capacity plus headroom for holes (agents removed
    // in a step occupy their slots until a binning drops them, or a birth of
    // a later step that keeps the binning takes the slot over)
    uint32_t capacity, slots, ncells, ntiles, n_init;
    // slots the agent-indexed kernels cover: all of them for a model with
    // children, else the capacity (without children the slots in use never
    // exceed it)
    uint32_t span;
    uint32_t tile_shift;         // a scan tile is kScanTile << tile_shift cells
    uint32_t birth_blocks;       // workgroups sorting birth runs (0: the model has no births)
    uint32_t n_sims;             // 1: a single simulation; tab has n_sims entries
    // launch shape of the neighbour search (performance only; results do
    // not depend on them): lanes per claimer (0: 4 for the 8-cell stencil,
    // 16 for the 27-cell one) and the fewest workgroups to launch
    uint32_t prop_lanes, prop_min_blocks;
    // claimer list: list_mode set (single simulations only) when the search
    // runs over the listed claimers instead of per chunk of sorted agents;
    // clist holds kListRegions regions of clist_cap entries, ccount their
    // counters (zeroed by finish for the next step); list_blocks workgroups
    // search
    uint32_t* clist;
    uint32_t* ccount;
    uint32_t clist_cap, list_mode, list_blocks;
};

// kernel indices for per-kernel timing
enum KernelId { kKMove = 0, kKScan, kKScatter, kKPropose, kKFinish, kNumKernels };
extern const char* const kKernelNames[kNumKernels];

// Optional start/stop events of a step kernel: when set, the dispatch itself
// timestamps them at the kernel's start and end (hipExtLaunchKernel), so the
// elapsed time is the kernel's own duration without the marker packets.
struct KEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// launch entry points (kernels.hip); each enqueues one kernel on `s`
void launch_init(const Dev& d, hipStream_t s);
// p: parity of the step (its agents start in a[p] and are sorted into
// a[p ^ 1]; for a step that keeps the binning the caller maps both to the
// buffer that holds the agents)
// bin = 0: the step keeps the previous step's cell lists (agents stay in
// their slots; move then sets the claimer flags and marks its removals as
// holes, there is no scan or scatter, and finish does the bookkeeping)
void launch_move(const Dev& d, int p, int record, int bin, uint32_t moved, hipStream_t s,
                 const KEvents& ev = {});
void launch_scan(const Dev& d, int p, hipStream_t s, const KEvents& ev = {});
void launch_scatter(const Dev& d, int p, int record, hipStream_t s, const KEvents& ev = {});
// moved: steps since the agents were binned (0 in a binning step)
void launch_propose(const Dev& d, int p, int bin, uint32_t moved, hipStream_t s,
                    const KEvents& ev = {});
void launch_finish(const Dev& d, int p, int record, int bin, hipStream_t s, const KEvents& ev = {});
// per-(simulation, species) live counts into d.counts, or into dst (same
// layout) with the step counter in *tslot (a counts-ring entry)
void launch_counts(const Dev& d, int cur, hipStream_t s, unsigned long long* dst = nullptr,
                   unsigned long long* tslot = nullptr);
void launch_fill_records(const Dev& d, hipStream_t s);
// per-simulation digests of the live agents (id, species, position bits)
// into out[n_sims] (verification queries)
void launch_digest(const Dev& d, int cur, unsigned long long* out, hipStream_t s);
// gathers simulation `sim`'s live agents into the birth records (id in
// parent, meta in sp), and with `record` their last-step cell ids and
// partners into bkey and events into `event`, counting them in
// ctl->export_n (queries between steps, when these arrays are free)
void launch_export(const Dev& d, int cur, uint32_t sim, int record, hipStream_t s);

}  // namespace mabm
