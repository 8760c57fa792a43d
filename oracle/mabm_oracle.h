/*
 * mabm_oracle.h -- plain, slow CPU oracle of the molecule-agent step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the HIP
 * library: it has its own Philox, its own log/sin/cos, its own cell list and
 * a brute-force neighbour mode.
 *
 * What it computes is the per-timestep update of the paper's molecule-level
 * agent-based simulator (Abstract; Sec. 2 "Materials and Methods"): every
 * molecule is an agent that diffuses in 3D, binds partners found by spatial
 * proximity, releases products, crosses compartments, is emitted by
 * expressors and degrades.  The paper leaves the stepping rules to earlier
 * work, so every rule below is a reading of the paper, written out phase by
 * phase (O0..O10) in mabm_oracle.c; each function names the phase it
 * implements.
 *
 * All floating point is IEEE binary32, evaluated left to right exactly as
 * written, built with -ffp-contract=off.
 */
#ifndef MABM_ORACLE_H
#define MABM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_STATE = -2, ORC_E_NOMEM = -3,
       ORC_E_CAPACITY = -4, ORC_E_DEVICE = -5 };
enum { ORC_PERIODIC_BOX = 0, ORC_SPHERE = 1, ORC_NESTED_SPHERES = 2 };
enum { ORC_BIMOL = 0, ORC_UNIMOL = 1 };
enum { ORC_KEEP = 0, ORC_SPLIT = 1, ORC_EMIT = 2, ORC_TRANSLOCATE = 3 };
enum { ORC_SEARCH_CELLS = 0, ORC_SEARCH_BRUTE = 1 };

typedef struct orc_sim orc_sim;

/* geometry: ORC_*; box_um: periodic cube side; outer/inner radius: spheres
 * centred at the origin (inner = nucleus, compartment 0, NESTED only).
 * grid_n: cells per axis of the exported cell id (0 = do not export ids). */
orc_sim* orc_create(int geometry, float box_um, float outer_radius_um,
                    float inner_radius_um, float dt_s, uint64_t seed,
                    uint32_t capacity, uint32_t grid_n);
void     orc_destroy(orc_sim* s);
const char* orc_last_error(const orc_sim* s);

int orc_add_species(orc_sim* s, float diffusion_um2_s, uint32_t initial_count,
                    int compartment);
int orc_add_rule(orc_sim* s, int kind, int r0, int r1, int p0, int p1,
                 float radius_um, double prob_per_step, int placement,
                 float release_radius_um, int from_comp, int to_comp);

/* neighbour search used by the propose phase: cell list or O(N^2) scan.
 * Both must give identical results; the brute-force mode is the pin. */
int orc_set_search(orc_sim* s, int mode);

/* Replace the initial placement by an explicit state (ids need not be
 * sorted; next_id must exceed every id).  t = step counter to resume at. */
int orc_import(orc_sim* s, uint32_t n, const uint32_t* id, const uint8_t* sp,
               const float* x, const float* y, const float* z,
               uint32_t next_id, uint32_t t);

int orc_step(orc_sim* s, uint32_t n_steps);
int orc_counts(orc_sim* s, uint64_t* out, uint32_t n_species, uint64_t* out_step);
/* number of live agents */
int orc_size(orc_sim* s, uint32_t* n, uint32_t* next_id);
/* live agents sorted by id.  key: cell id of the moved position in the
 * last step (0xFFFFFFFF if none); event: unimolecular rule fired in the last
 * step (-1 none); partner: id of the confirmed partner in the last step
 * (0xFFFFFFFF none).  Any output pointer may be NULL. */
int orc_export(orc_sim* s, uint32_t cap, uint32_t* id, uint8_t* sp, float* x,
               float* y, float* z, uint32_t* key, int32_t* event,
               uint32_t* partner);

/* ---- building blocks exposed for the pin tests ---- */
void  orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_log(float x);
void  orc_sincos2pi(float a, float* s, float* c);
/* the three N(0,1) draws of the Brownian move of agent id at step t */
void  orc_gauss3(uint64_t seed, uint32_t id, uint32_t t, float out[3]);
/* the 32-bit unimolecular event draw of agent id at step t */
uint32_t orc_event_word(uint64_t seed, uint32_t id, uint32_t t);
/* threads of the parallel per-agent loops (n > 0 sets them); returns the
 * count the next step uses */
int orc_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
