/*
 * mabm.h -- C ABI of the MI355X (gfx950) molecule-agent step library.
 *
 * The library advances a molecule-level agent-based simulation of a
 * signalling pathway (Maestri, "Towards In Silico Cancer Therapy Design",
 * Abstract and Sec. 2): every molecule is an agent with a species, an id and
 * a position in a 3D volume.  One step moves every agent by a Brownian
 * displacement, finds reaction partners by spatial proximity, fires binding,
 * catalysis, unbinding, translocation, emission and degradation rules, and
 * compacts births and deaths.  The exact step definition (random-number
 * layout, boundaries, claim rule, placement of products) is fixed in phases
 * O0..O10, the same for this library and for the oracle its tests compare
 * it with.  Every call below names the paper passage whose input or output
 * it carries; the calls that are infrastructure of a C library (freeing a
 * handle, error messages, timing, launch parameters) say "no passage".
 *
 * Conventions for every call:
 *   - Return value: mabm_status, 0 = MABM_OK, negative = error.  No call
 *     aborts or throws; mabm_last_error() gives a message.
 *   - Pointers named device_* are HIP device pointers; every other pointer
 *     is host memory owned by the caller and only read/written during the
 *     call.
 *   - Device memory: the library allocates none.  The caller passes one
 *     device arena of at least mabm_arena_bytes() bytes and a HIP stream;
 *     both are borrowed and must outlive the simulation.
 *   - Steps are enqueued asynchronously on the stream; mabm_counts and
 *     mabm_export synchronise it.  Device-side failures (capacity overflow,
 *     placement failure) are sticky: they are reported by the next
 *     synchronising call, after which only mabm_destroy_sim and
 *     mabm_last_error are valid.
 *   - One simulation must not be used from two host threads at once;
 *     distinct simulations are independent.
 */
#ifndef MABM_H
#define MABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MABM_ABI_VERSION 1u
#define MABM_MAX_SPECIES 64
#define MABM_MAX_RULES 255
/* Cells per axis of the spatial hash, at most (a finer cell_um is coarsened
 * to it); the grids of one handle's simulations hold at most 2^31 cells
 * together, counted at the power of two at or above each grid (else
 * E_INVALID, and mabm_arena_bytes returns 0). */
#define MABM_MAX_GRID 1024
#define MABM_NONE 0xFFFFFFFFu

typedef enum {
    MABM_OK = 0,
    MABM_E_INVALID = -1,  /* bad argument or inconsistent model            */
    MABM_E_STATE = -2,    /* call not allowed in this state                 */
    MABM_E_NOMEM = -3,    /* arena too small                                */
    MABM_E_CAPACITY = -4, /* more live agents (or births) than the capacity */
    MABM_E_DEVICE = -5    /* HIP runtime error or device-side failure       */
} mabm_status;

/* Simulated volume (Sec. 2 footnote: simulation volume, compartments).
 * PERIODIC_BOX: cube [0, box_um)^3 with periodic wrap, one compartment 0.
 * SPHERE: ball of outer_radius_um at the origin, one compartment 0.
 * NESTED_SPHERES: nucleus (compartment 0, |p| < inner_radius_um) inside a
 * cell (compartment 1, inner <= |p| <= outer_radius_um). */
typedef enum { MABM_PERIODIC_BOX = 0, MABM_SPHERE = 1, MABM_NESTED_SPHERES = 2 } mabm_geometry;

typedef enum { MABM_BIMOL = 0, MABM_UNIMOL = 1 } mabm_rule_kind;

/* Placement of a rule's products (Abstract: binding, release of reaction
 * products, migration between compartments; Sec. 2: expressors).
 * KEEP: products replace the reactants in place (binding, catalysis,
 *       conversion, degradation when the product is -1).
 * SPLIT: unimolecular A -> P1 + P2, P1 at p+u and P2 at p-u, u uniform in
 *       the ball of release_radius_um (unbinding).
 * EMIT: unimolecular A -> A (or P1) + child P2 at p+u (expression).
 * TRANSLOCATE: unimolecular crossing of the nuclear membrane from from_comp
 *       to to_comp, landing release_radius_um across it, radially. */
typedef enum { MABM_KEEP = 0, MABM_SPLIT = 1, MABM_EMIT = 2, MABM_TRANSLOCATE = 3 } mabm_placement;

typedef struct {
    uint32_t abi_version;  /* MABM_ABI_VERSION */
    int32_t geometry;      /* mabm_geometry */
    float box_um;          /* PERIODIC_BOX side, um */
    float outer_radius_um; /* SPHERE / NESTED_SPHERES outer radius, um */
    float inner_radius_um; /* NESTED_SPHERES nucleus radius, um */
    float dt_s;            /* time step, s (> 0) */
    uint64_t seed;         /* Philox key */
    uint32_t capacity;     /* maximum live agents at any step end (see below) */
    float cell_um;         /* spatial-hash cell size, um; 0 = chosen by the library;
                              at most MABM_MAX_GRID cells per axis */
    uint32_t flags;        /* MABM_FLAG_* */
} mabm_config;

/* Capacity.  A step whose end leaves more live agents than the capacity
 * (births and removals of that step counted as the step definition's
 * compaction counts them) makes the simulation fail with E_CAPACITY,
 * reported by the next synchronising call, exactly at the step where the
 * definition overflows, whatever the binning interval.  Agents removed in a
 * step keep their array slots until a binning compacts them, or until a
 * child of a later step that keeps the binning takes the slot over, so the
 * agent arrays hold the capacity plus a quarter more (mabm_arena_bytes
 * includes it); only a step whose pair rules remove more than that quarter
 * while the live agents are near the capacity runs out of slots, which is
 * E_CAPACITY too, with its own message.  A step's children are not
 * otherwise limited (up to one per live agent). */

/* Record, for every live agent, the cell id, unimolecular event and partner
 * of the last step, so that mabm_export can return them.  Costs extra
 * traffic; results are identical with and without it. */
#define MABM_FLAG_RECORD 1u
/* Launch each step's kernels directly instead of replaying a captured HIP
 * graph (graphs are used only on a non-null stream and without per-kernel
 * timing).  Results are identical either way. */
#define MABM_FLAG_NO_GRAPH 2u

/* Per-step rule (Sec. 2: "reactions it participates in, including
 * interacting partners, rates, and resulting products").  Species are ids
 * returned by mabm_add_species; -1 = none.
 * BIMOL: reactant[0] is the claimer, reactant[1] the target; on contact
 *   (centre distance <= radius_um, same compartment) the pair fires with
 *   probability prob_per_step; claimer -> product[0], target -> product[1]
 *   (-1 = the agent is consumed).  placement must be KEEP.  At most one
 *   BIMOL rule per unordered species pair.
 * UNIMOL: reactant[0] fires with probability prob_per_step per step when in
 *   from_comp (-1 = any compartment); the probabilities of one species'
 *   rules in one compartment must sum to <= 1. */
typedef struct {
    int32_t kind;             /* mabm_rule_kind */
    int32_t reactant[2];
    int32_t product[2];
    float radius_um;          /* BIMOL contact radius */
    double prob_per_step;     /* in [0, 1] */
    int32_t placement;        /* mabm_placement */
    float release_radius_um;  /* SPLIT/EMIT ball radius; TRANSLOCATE offset (>= 1e-3) */
    int32_t from_comp, to_comp;
} mabm_rule;

/* Device bytes a simulation with this configuration needs (an upper bound
 * independent of the model's species and rules beyond the stated counts).
 * Passage: Sec. 3.2 -- the multiple-seed runs were throughput-bound, many
 * seeds sharing one GPU; the footprint is what a scheduler admits such runs
 * by.  Returns 0 for an invalid config. */
size_t mabm_arena_bytes(const mabm_config* cfg, uint32_t n_species, uint32_t n_rules);

/* Create a simulation in the caller's device arena, working on the caller's
 * HIP stream (a hipStream_t, NULL = the null stream).  Passage: Sec. 2,
 * footnote on the key parameters -- the simulation volume and, for models
 * with compartments, the compartments (here the geometry and its radii);
 * the seed keys the random draws (Sec. 3.3 reports runs over several
 * seeds).  The arena is carved,
 * not cleared beyond what the library needs.  *out receives an opaque handle
 * owned by the caller (free with mabm_destroy_sim).
 * Errors: E_INVALID (config), E_NOMEM (arena_bytes too small), E_DEVICE. */
typedef struct mabm_sim mabm_sim;
mabm_status mabm_create_sim(const mabm_config* cfg, void* device_arena, size_t arena_bytes,
                            void* hip_stream, mabm_sim** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): create a
 * simulation like mabm_create_sim, but in the library's static arena on
 * the current device instead of a caller's arena.  The arena is a
 * file-scope device array of 64 MiB (2^26 bytes) per device, held by every
 * device the library runs on until the process ends; a configuration whose
 * mabm_arena_bytes exceeds it is rejected with E_NOMEM.  The call allocates
 * no device memory (no hipMalloc or allocating library routine), and the
 * simulation's steps run as direct kernel launches, never as graphs (the
 * MABM_FLAG_NO_GRAPH flag is forced), so stepping it allocates none either.
 * One device's arena holds one simulation at a time: a second call on the
 * device before mabm_destroy_sim of the first returns E_STATE.  The arena
 * keeps the last simulation's contents; everything a simulation needs
 * cleared is cleared when its model is finalized.  Host threads that use
 * the arena of one device must not overlap (they would race on it).
 * Other arguments, ownership and errors as mabm_create_sim. */
mabm_status mabm_create_sim_static(const mabm_config* cfg, void* hip_stream, mabm_sim** out);

/* Add a species (Sec. 2: molecular species with diffusion from
 * Stokes-Einstein, initial concentration -> count, localisation ->
 * compartment).  Ids 0, 1, ... in call order.  E_STATE after the model is
 * finalized (first step/counts/export/import). */
mabm_status mabm_add_species(mabm_sim* sim, const char* name, float diffusion_um2_s,
                             uint32_t initial_count, int32_t compartment, int32_t* out_species_id);

/* Add a rule; validated at once (unknown species, probability outside
 * [0,1], bad placement or compartments, a second BIMOL rule for a pair:
 * E_INVALID).  Ids 0, 1, ... in call order. */
mabm_status mabm_add_rule(mabm_sim* sim, const mabm_rule* rule, int32_t* out_rule_id);

/* Cells per axis and cell size the simulation uses (after finalize).  No
 * passage: the spatial hash is this library's own device. */
mabm_status mabm_grid(mabm_sim* sim, uint32_t* cells_per_axis, float* cell_um);

/* Enqueue n_steps steps on the stream; returns without synchronising.  The
 * first call finalizes the model: consistency checks of Sec. 2 (probability
 * sums, radii against the cell size: E_INVALID), table upload and initial
 * placement. */
mabm_status mabm_step(mabm_sim* sim, uint32_t n_steps);

/* Per-species counts of live agents after the last enqueued step (Sec. 2:
 * concentrations over time; out has n_species entries) and the step
 * counter.  Synchronises the stream; reports sticky device errors. */
mabm_status mabm_counts(mabm_sim* sim, uint64_t* out, uint32_t n_species, uint64_t* out_step);

/* Number of live agents and the next id to be assigned (synchronises).
 * Passage: Sec. 2, each molecule is an agent; the live count is the
 * population the concentrations of Sec. 2 are taken over. */
mabm_status mabm_size(mabm_sim* sim, uint32_t* n_live, uint32_t* next_id);

/* Copy the live agents to host arrays of capacity >= n_live, sorted by id.
 * Passage: Sec. 2, the three-dimensional viewer of the agents' spatial
 * dynamics -- this is the state such a view (or a checkpoint) reads.
 * key: cell id cx + G (cy + G cz) of the moved position in the last step;
 * event: unimolecular rule fired in the last step (-1 none); partner: id of
 * the confirmed partner in the last step (MABM_NONE none).  key, event and
 * partner need MABM_FLAG_RECORD (else MABM_NONE / -1).  Any pointer may be
 * NULL.  Synchronises. */
mabm_status mabm_export(mabm_sim* sim, uint32_t capacity, uint32_t* id, uint8_t* species,
                        float* x, float* y, float* z, uint32_t* key, int32_t* event,
                        uint32_t* partner);

/* Passage: Sec. 2, per-species localisation and initial concentrations
 * given by the user instead of the library's uniform placement (and Sec.
 * 3.2's long runs, resumed from a checkpoint).
 * Replace the initial placement (or resume a checkpoint): n agents with the
 * given ids (distinct, all < next_id), species and positions (inside the
 * volume), and the step counter t.  E_INVALID for a null array (n > 0), an
 * unknown species, a repeated id, an id not below next_id or a position
 * outside the volume; E_CAPACITY for n above the capacity; E_STATE after
 * the model was finalized or on a batch.  Finalizes the model.
 * Synchronises. */
mabm_status mabm_import(mabm_sim* sim, uint32_t n, const uint32_t* id, const uint8_t* species,
                        const float* x, const float* y, const float* z, uint32_t next_id,
                        uint32_t t);

/* ------------------------------------------------------------------------
 * Batches: many independent simulations of one model stepped together.
 *
 * A dose x replicate sweep runs the same species and rules many times with
 * different seeds, volume sizes and initial counts (the paper's dose-response
 * study, Sec. 3.1, and its multiple-seed runs, Sec. 3.2).  A batch holds
 * n_sims such simulations in one arena; every step is one set of kernel
 * launches over all their agents (cells of different simulations never
 * meet), so small simulations no longer pay the launch latency one by one.
 * Each simulation's trajectory is identical, bit for bit, to the one
 * mabm_create_sim gives for its configuration and counts.
 *
 * The configurations must agree on geometry, dt_s and flags; seed, volume
 * size, capacity and cell size may differ; 1 <= n_sims <= 65535 and the
 * summed capacity is at most 2^30.  On a batch handle, mabm_add_species,
 * mabm_add_rule and mabm_step act on every simulation; mabm_add_species's
 * initial_count applies to all of them until mabm_set_initial_counts sets
 * one count per simulation; mabm_counts returns the per-species totals over
 * the batch; mabm_grid gives simulation 0's grid; mabm_size, mabm_export and
 * mabm_import are E_STATE (use the mabm_batch_* calls).  Each simulation's
 * capacity holds for it alone (E_CAPACITY names the first simulation that
 * overflowed); the slots are pooled.
 * ---------------------------------------------------------------------- */

/* Device bytes of a batch (0 if the configurations are invalid or
 * inconsistent); mabm_arena_bytes(cfg, ...) equals it with n_sims = 1. */
size_t mabm_batch_arena_bytes(const mabm_config* cfgs, uint32_t n_sims, uint32_t n_species,
                              uint32_t n_rules);

/* Create a batch of n_sims simulations (cfgs[k] for simulation k) in one
 * device arena, on one HIP stream; same ownership and errors as
 * mabm_create_sim. */
mabm_status mabm_create_batch(const mabm_config* cfgs, uint32_t n_sims, void* device_arena,
                              size_t arena_bytes, void* hip_stream, mabm_sim** out);

/* Initial counts of one species, one per simulation (counts has n_sims
 * entries; Sec. 3.1's doses are initial inhibitor counts).  Before
 * finalize; E_INVALID for an unknown species. */
mabm_status mabm_set_initial_counts(mabm_sim* sim, int32_t species_id, const uint32_t* counts);

/* Per-(simulation, species) live counts: out[k * n_species + s] for
 * simulation k; out has n_sims * n_species entries.  Synchronises. */
mabm_status mabm_batch_counts(mabm_sim* sim, uint64_t* out, uint32_t n_species,
                              uint64_t* out_step);

/* mabm_size, mabm_export and mabm_grid of simulation sim_index (also valid
 * on a single simulation with sim_index 0).  E_INVALID for an index out of
 * range. */
mabm_status mabm_batch_size(mabm_sim* sim, uint32_t sim_index, uint32_t* n_live,
                            uint32_t* next_id);
mabm_status mabm_batch_export(mabm_sim* sim, uint32_t sim_index, uint32_t capacity, uint32_t* id,
                              uint8_t* species, float* x, float* y, float* z, uint32_t* key,
                              int32_t* event, uint32_t* partner);
mabm_status mabm_batch_grid(mabm_sim* sim, uint32_t sim_index, uint32_t* cells_per_axis,
                            float* cell_um);

/* Counts over time without host synchronisation (Sec. 2: species are
 * monitored against concentration thresholds within time windows; Sec. 3.2
 * names step-wise host-device synchronisation and periodic output among the
 * original simulator's costs).  While every > 0, after each step whose
 * number since the first step is a multiple of every, the library appends
 * one entry to a ring in the caller's device memory (device_ring, entries x
 * mabm_ring_entry_bytes(sim) bytes, 8-byte aligned, borrowed until the ring
 * is switched off with every = 0); a full ring overwrites its oldest entry.
 * An entry is uint64 words: the step counter, then for every simulation of
 * the handle (one unless it is a batch) MABM_MAX_SPECIES species counts.
 * Recording splits graph replays at entry steps; results do not change.
 * Replacing a ring, or switching it off, first synchronises the stream, so
 * the old buffer may be freed (or reused) as soon as the call returns; the
 * new buffer must be ready (e.g. zero-filled) before the stream's next
 * step, i.e. filled on that stream or on one it waits for. */
size_t mabm_ring_entry_bytes(const mabm_sim* sim);
mabm_status mabm_counts_ring(mabm_sim* sim, void* device_ring, uint32_t entries, uint32_t every);

/* Copy the newest min(recorded, entries, max_entries) ring entries, oldest
 * first, to out (max_entries x mabm_ring_entry_bytes bytes); *n_recorded
 * receives the number of entries recorded since the ring was set.
 * Synchronises the stream. */
mabm_status mabm_ring_read(mabm_sim* sim, uint64_t* out, uint32_t max_entries,
                           uint64_t* n_recorded);

/* No passage (tuning of this library's kernels).
 * Launch-shape parameters of the neighbour search, for tuning (results do
 * not depend on them).  MABM_PARAM_PROPOSE_LANES: lanes per claimer, 4, 8,
 * 16 or 32 (0: the library's choice; raised to the least that covers the
 * stencil with two cells per lane).  MABM_PARAM_PROPOSE_MIN_WORKGROUPS: the
 * fewest workgroups (of 256 threads, one per chunk of 1,024 sorted agents)
 * the search launches, chunks being shared by up to 16 workgroups to reach
 * it (0: 2048).  Synchronises the
 * stream; E_INVALID for an unknown parameter or value. */
#define MABM_PARAM_PROPOSE_LANES 1
#define MABM_PARAM_PROPOSE_MIN_WORKGROUPS 2
/* MABM_PARAM_BIN_EVERY_MAX: the most steps between two binnings of the
 * agents into cells (0: the library's limit, 8; 1: every step).  Between
 * binnings agents keep their array slots and the neighbour search reads the
 * last binning's cell lists (agents that rules place since the binning are
 * listed apart); the library bins only as rarely as keeps every result
 * unchanged (every contact radius plus the largest possible Brownian moves
 * since the binning within the stencil's reach), and every step for models
 * without pair rules.  Results do not depend on it. */
#define MABM_PARAM_BIN_EVERY_MAX 3
/* MABM_PARAM_BIN_EVERY (mabm_get_param only): steps between binnings in
 * effect (finalizes the model). */
#define MABM_PARAM_BIN_EVERY 4
/* MABM_PARAM_PROPOSE_MODE: how the neighbour search finds the claimers
 * (results do not depend on it).  1: per chunk of 1,024 agents in cell
 * order, a workgroup searching the chunk's claimers with 4 lanes each (16
 * for the 27-cell stencil).  2: over a list of the step's claimers, built by
 * the kernel that flags them, every claimer getting 16 to 64 lanes as the
 * list's length allows and a stencil cell's candidates shared by several of
 * them (for sparse claimers in crowded cells); single simulations only
 * (E_INVALID for a batch).  0 (default): 2 for a single simulation whose
 * claimer species hold under 1/64 of its initial agents or at most 32,768
 * of them, else 1.
 * mabm_get_param returns the mode in use, 1 or 2 (finalizes the model). */
#define MABM_PARAM_PROPOSE_MODE 5
mabm_status mabm_set_param(mabm_sim* sim, int32_t param, uint32_t value);
mabm_status mabm_get_param(mabm_sim* sim, int32_t param, uint32_t* value);

/* No passage (measurement of this library's kernels).
 * Per-kernel timing: while enabled (1), each step kernel is dispatched with
 * a pair of HIP events that the dispatch itself stamps at the kernel's start
 * and end, so the time is the kernel's own duration; steps then run as
 * direct launches, somewhat slower than untimed ones.  Disable with 0.  read
 * returns, per kernel of the step, the number of launches timed and their
 * total milliseconds (synchronises); names receives a static string per
 * kernel. */
#define MABM_N_KERNELS 5
mabm_status mabm_profile(mabm_sim* sim, int32_t enable);
mabm_status mabm_profile_read(mabm_sim* sim, const char** names, uint64_t* launches,
                              double* total_ms);

/* Sum over all steps so far of the live agents at the start of each step
 * (the agent-update count).  Passage: Sec. 3.2, per-step cost scales with
 * the agent count; this is that count summed over the steps run.
 * Synchronises. */
mabm_status mabm_agent_updates(mabm_sim* sim, uint64_t* out);

/* Digest of the current state, one per simulation of the handle (out has
 * n = 1 entry, or n_sims for a batch): the sum mod 2^64 over the live agents
 * of a 64-bit hash of (id, species, position bits), mixed by MurmurHash3's
 * 64-bit finaliser as h = f(f(f((id << 32 | species) ^ 0x9E3779B97F4A7C15)
 * ^ (x_bits << 32 | y_bits)) ^ z_bits).  It does not depend on where the
 * agents sit in memory, so two runs that reach the same id-keyed state give
 * the same digest, and a state that differs in any agent's id, species or
 * position bits gives another one with overwhelming probability.  No
 * passage (verification: checking that batched and served runs equal
 * single runs without copying whole states to the host).  E_INVALID if n is
 * not the handle's simulation count.  Synchronises. */
mabm_status mabm_digest(mabm_sim* sim, uint64_t* out, uint32_t n);

/* Free the host handle (the arena and stream stay the caller's).  No
 * passage (C library infrastructure). */
mabm_status mabm_destroy_sim(mabm_sim* sim);

/* Message of the last failing call on sim (or of the last failed create
 * when sim is NULL).  Valid until the next call on sim.  No passage (C
 * library infrastructure); the messages of model errors name the
 * consistency checks of Sec. 2. */
const char* mabm_last_error(const mabm_sim* sim);

#ifdef __cplusplus
}
#endif
#endif /* MABM_H */
