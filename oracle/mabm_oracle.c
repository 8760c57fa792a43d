/*
 * mabm_oracle.c -- plain CPU oracle of the molecule-agent step.
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It is deliberately slow and literal:
 * one loop per phase of the step definition, in the order the phases are
 * defined, no blocking, no fusion.  The two per-agent loops whose
 * iterations are independent (the move phase, where each agent writes only
 * its own fields and appends at most one child, and the neighbour search of
 * each claimer) are shared among OpenMP threads; children are ordered by
 * parent id before they get ids, so no result depends on the thread count
 * (a test compares 1 thread with several).
 *
 * Paper: the simulator of Maestri, "Towards In Silico Cancer Therapy Design"
 * (Abstract; Sec. 2).  Molecules are agents with physical properties that
 * diffuse in a 3D volume (Sec. 2, diffusion from Stokes-Einstein), interact
 * by spatial proximity (Sec. 2, first paragraph), bind and release reaction
 * products (Abstract), migrate between compartments (Abstract; Sec. 3.4) and
 * are emitted by expressor agents (Sec. 2, functional classes) or degraded
 * (Sec. 3.4).  The paper defers the exact stepping rules to earlier work, so
 * the step is fixed by a definition in phases O0..O10; the comment of each
 * function states the phase it follows and the reading it takes where the
 * paper is silent.
 *
 * Parity pins: Philox against rocRAND's host implementation; log/sin/cos
 * against numpy float64; neighbour search against the O(N^2) mode; the
 * stochastic laws (MSD = 6Dt, A+B<->C detailed balance, binomial decay,
 * two-state translocation, uniform placement) in tests/test_oracle_*.py.
 */
#include "mabm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXS 64
#define MAXR 256
#define MAXU 8
#define NONE32 0xFFFFFFFFu

/* Philox counter "purpose" words (third counter word). */
/* (word 1 is not used: the event draw shares the MOVE block, see O2) */
enum { PUR_INIT = 0, PUR_MOVE = 2, PUR_PAIR = 3, PUR_PRIO = 4, PUR_BIRTH = 5 };

typedef struct {
    int kind, r0, r1, p0, p1, placement, from, to;
    float radius, r2, release, release2, target_r;
    double prob;
    uint64_t thr; /* bimolecular Bernoulli threshold, in [0, 2^32] */
} rule_t;

typedef struct {
    uint32_t parent;
    uint8_t sp;
    float x, y, z;
} child_t;

struct orc_sim {
    int geometry, ncomp;
    float L, halfL, Rout, Rout2, Rin, Rin2, dt;
    uint64_t seed;
    uint32_t pkey[2];
    uint32_t capacity, grid_n;
    float grid_lo, grid_inv_h;

    int ns, nr;
    float D[MAXS];
    uint32_t init_count[MAXS];
    int init_comp[MAXS];
    float sigma[MAXS];
    rule_t rule[MAXR];
    int uni_n[MAXS][2];
    int uni_rule[MAXS][2][MAXU];
    uint64_t uni_thr[MAXS][2][MAXU];
    int rule_of[MAXS][MAXS];
    int is_claimer[MAXS];
    float rmax;

    int tables_ready, placed, failed, search;
    uint32_t t, next_id, n;

    /* state (array order is irrelevant to every result) */
    uint32_t* id;
    uint8_t* sp;
    float *x, *y, *z;

    /* per-step scratch, indexed like the state */
    float *mx, *my, *mz;  /* moved position p' */
    float *fx, *fy, *fz;  /* final position    */
    uint8_t* fsp;         /* final species     */
    uint8_t* alive;       /* survives the step */
    uint8_t* busy;        /* has a unimolecular event: takes no part in pairing */
    int32_t* event;
    uint32_t* key;
    uint32_t* partner;
    int32_t* prop_b;
    int32_t* prop_r;
    uint64_t* slot;
    child_t* kids;
    uint32_t nkids;

    /* oracle's own cell list for the propose phase */
    uint32_t og;
    float olo, oinv;
    int32_t* head;
    int32_t* nxt;

    char err[256];
};

static int fail(orc_sim* s, int code, const char* msg)
{
    snprintf(s->err, sizeof s->err, "%s", msg);
    return code;
}

/* ------------------------------------------------------------------------
 * O1: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter of four
 * 32-bit words, key of two; ten rounds, the key bumped by the two Weyl
 * constants between rounds.  Each round multiplies words 0 and 2 by the two
 * round multipliers and recombines high/low halves with words 1, 3 and the
 * key.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t a_hi = (uint32_t)(a >> 32), a_lo = (uint32_t)a;
        uint32_t b_hi = (uint32_t)(b >> 32), b_lo = (uint32_t)b;
        uint32_t n0 = b_hi ^ c1 ^ k0;
        uint32_t n1 = b_lo;
        uint32_t n2 = a_hi ^ c3 ^ k1;
        uint32_t n3 = a_lo;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw_k(const uint32_t key[2], uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                   uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    orc_philox4x32_10(ctr, key, out);
}

static void draw(const orc_sim* s, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t out[4])
{
    draw_k(s->pkey, c0, c1, c2, c3, out);
}

/* O1: 24-bit uniforms.  u in [0,1), u_plus in (0,1]; both exact in float. */
static float unif(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
static float unif_plus(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }

/* ------------------------------------------------------------------------
 * O3 helper: natural logarithm for x in (0, 1].  x = m * 2^e with m folded
 * into (sqrt(1/2), sqrt(2)]; log m = 2 atanh(s), s = (m-1)/(m+1), summed as
 * the Maclaurin series of atanh up to s^9 (|s| < 0.172, so the first
 * omitted term, s^11/11, is below 4e-10 relative) by Horner's rule with
 * fused multiply-adds.  ln 2 is split into a 16-bit head, exact when
 * multiplied by the small exponent, plus the float nearest the remainder.
 * ---------------------------------------------------------------------- */
float orc_log(float x)
{
    const float SQRT2 = 0x1.6a09e6p+0f;      /* float nearest sqrt(2) */
    const float LN2_HEAD = 0x1.62e4p-1f;     /* ln 2 rounded to 16 bits */
    const float LN2_TAIL = 0x1.7f7d1cp-20f;  /* float nearest ln 2 - head */
    uint32_t bits;
    memcpy(&bits, &x, 4);
    int e = (int)((bits >> 23) & 0xffu) - 127;
    uint32_t mbits = (bits & 0x7fffffu) | 0x3f800000u;
    float m;
    memcpy(&m, &mbits, 4);
    if (m > SQRT2) {
        m = m * 0.5f;
        e = e + 1;
    }
    float s = (m - 1.0f) / (m + 1.0f);
    float s2 = s * s;
    float q = 1.0f / 9.0f;
    q = fmaf(q, s2, 1.0f / 7.0f);
    q = fmaf(q, s2, 1.0f / 5.0f);
    q = fmaf(q, s2, 1.0f / 3.0f);
    q = q * s2;
    float lm = fmaf(s, q, s) * 2.0f;
    float fe = (float)e;
    return fmaf(fe, LN2_HEAD, fmaf(fe, LN2_TAIL, lm));
}

/* ------------------------------------------------------------------------
 * O3 helper: sin and cos of 2*pi*a for a in [0, 1) on the 2^-24 grid.
 * Quadrant q = floor(4a) and remainder r = 4a - q are exact; r > 1/2 is
 * folded to 1 - r (exact) with sin and cos swapped; x = r * (pi/2) lies in
 * [0, pi/4], where the Maclaurin series of sin (to x^9) and cos (to x^8)
 * are summed by Horner's rule with fused multiply-adds and coefficients
 * +-1/n! (first omitted terms below 2e-9 and 5e-8 at pi/4).
 * ---------------------------------------------------------------------- */
void orc_sincos2pi(float a, float* out_s, float* out_c)
{
    const float PI_2 = 0x1.921fb6p+0f; /* float nearest pi/2 */
    float a4 = a * 4.0f;
    int q = (int)a4;
    float r = a4 - (float)q;
    int fold = r > 0.5f;
    if (fold) r = 1.0f - r;
    float x = r * PI_2;
    float x2 = x * x;
    float ps = 1.0f / 362880.0f;
    ps = fmaf(ps, x2, -(1.0f / 5040.0f));
    ps = fmaf(ps, x2, 1.0f / 120.0f);
    ps = fmaf(ps, x2, -(1.0f / 6.0f));
    ps = ps * x2;
    float sx = fmaf(x, ps, x);
    float pc = 1.0f / 40320.0f;
    pc = fmaf(pc, x2, -(1.0f / 720.0f));
    pc = fmaf(pc, x2, 1.0f / 24.0f);
    pc = fmaf(pc, x2, -0.5f);
    float cx = fmaf(pc, x2, 1.0f);
    float s1 = fold ? cx : sx;
    float c1 = fold ? sx : cx;
    switch (q & 3) {
    case 0: *out_s = s1; *out_c = c1; break;
    case 1: *out_s = c1; *out_c = -s1; break;
    case 2: *out_s = -s1; *out_c = -c1; break;
    default: *out_s = -c1; *out_c = s1; break;
    }
}

/* O2/O3: the Philox block (id, t, MOVE) of one agent and step.  Its four
 * high 24-bit fields feed Box-Muller; its four low bytes, word 0 lowest,
 * form the 32-bit event draw. */
static void move_block(const uint32_t key[2], uint32_t id, uint32_t t, uint32_t w[4])
{
    draw_k(key, id, t, PUR_MOVE, 0, w);
}

static uint32_t event_word(const uint32_t w[4])
{
    return (w[0] & 0xFFu) | ((w[1] & 0xFFu) << 8) | ((w[2] & 0xFFu) << 16) | ((w[3] & 0xFFu) << 24);
}

/* O3: three N(0,1) draws by Box-Muller from the MOVE block. */
static void gauss3_w(const uint32_t w[4], float z[3])
{
    float r1 = sqrtf(-2.0f * orc_log(unif_plus(w[0])));
    float sn, cs;
    orc_sincos2pi(unif(w[1]), &sn, &cs);
    z[0] = r1 * cs;
    z[1] = r1 * sn;
    float r2 = sqrtf(-2.0f * orc_log(unif_plus(w[2])));
    orc_sincos2pi(unif(w[3]), &sn, &cs);
    z[2] = r2 * cs;
}

void orc_gauss3(uint64_t seed, uint32_t id, uint32_t t, float out[3])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, w[4];
    move_block(key, id, t, w);
    gauss3_w(w, out);
}

uint32_t orc_event_word(uint64_t seed, uint32_t id, uint32_t t)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, w[4];
    move_block(key, id, t, w);
    return event_word(w);
}

/* ------------------------------------------------------------------------
 * Geometry (O4).  Compartment 0 is the inner sphere (nucleus) of the nested
 * geometry, membership strict: |p|^2 < R_in^2.  Single-volume geometries
 * have one compartment, 0.
 * ---------------------------------------------------------------------- */
static float norm2(float x, float y, float z) { return x * x + y * y + z * z; }

static int comp_of(const orc_sim* s, float x, float y, float z)
{
    if (s->geometry != ORC_NESTED_SPHERES) return 0;
    return norm2(x, y, z) < s->Rin2 ? 0 : 1;
}

static float wrap1(const orc_sim* s, float v)
{
    if (v < 0.0f) v += s->L;
    if (v >= s->L) v -= s->L;
    return v;
}

/* inside the simulated volume and in compartment c (box: always) */
static int valid_at(const orc_sim* s, float x, float y, float z, int c)
{
    if (s->geometry == ORC_PERIODIC_BOX) return 1;
    float n2 = norm2(x, y, z);
    if (n2 > s->Rout2) return 0;
    if (s->geometry == ORC_NESTED_SPHERES && (n2 < s->Rin2 ? 0 : 1) != c) return 0;
    return 1;
}

/* O6: exported cell id of a position: linear index cx + G (cy + G cz) of
 * the grid of G cells per axis over the bounding box. */
static uint32_t cell_axis(float v, float lo, float inv_h, uint32_t g)
{
    float f = floorf((v - lo) * inv_h);
    if (!(f >= 0.0f)) return 0;
    if (f >= (float)g) return g - 1;
    return (uint32_t)f;
}

static uint32_t export_key(const orc_sim* s, float x, float y, float z)
{
    uint32_t g = s->grid_n;
    if (g == 0) return NONE32;
    uint32_t cx = cell_axis(x, s->grid_lo, s->grid_inv_h, g);
    uint32_t cy = cell_axis(y, s->grid_lo, s->grid_inv_h, g);
    uint32_t cz = cell_axis(z, s->grid_lo, s->grid_inv_h, g);
    return cx + g * (cy + g * cz);
}

/* ------------------------------------------------------------------------ */
orc_sim* orc_create(int geometry, float box_um, float outer_radius_um, float inner_radius_um,
                    float dt_s, uint64_t seed, uint32_t capacity, uint32_t grid_n)
{
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->geometry = geometry;
    s->L = box_um;
    s->halfL = box_um * 0.5f;
    s->Rout = outer_radius_um;
    s->Rin = inner_radius_um;
    s->Rout2 = (float)((double)outer_radius_um * (double)outer_radius_um);
    s->Rin2 = (float)((double)inner_radius_um * (double)inner_radius_um);
    s->dt = dt_s;
    s->seed = seed;
    s->pkey[0] = (uint32_t)seed;
    s->pkey[1] = (uint32_t)(seed >> 32);
    s->capacity = capacity;
    s->grid_n = grid_n;
    s->ncomp = geometry == ORC_NESTED_SPHERES ? 2 : 1;
    if (geometry == ORC_PERIODIC_BOX) {
        s->grid_lo = 0.0f;
        s->grid_inv_h = grid_n ? (float)((double)grid_n / (double)box_um) : 0.0f;
    } else {
        s->grid_lo = -outer_radius_um;
        s->grid_inv_h = grid_n ? (float)((double)grid_n / (2.0 * (double)outer_radius_um)) : 0.0f;
    }
    for (int a = 0; a < MAXS; ++a)
        for (int b = 0; b < MAXS; ++b) s->rule_of[a][b] = -1;
    int bad = 0;
    if (geometry < 0 || geometry > 2) bad = 1;
    if (geometry == ORC_PERIODIC_BOX && !(box_um > 0.0f)) bad = 1;
    if (geometry != ORC_PERIODIC_BOX && !(outer_radius_um > 0.0f)) bad = 1;
    if (geometry == ORC_NESTED_SPHERES &&
        !(inner_radius_um > 0.0f && inner_radius_um < outer_radius_um))
        bad = 1;
    if (!(dt_s > 0.0f) || capacity == 0) bad = 1;
    size_t c = capacity;
    s->id = malloc(c * 4); s->sp = malloc(c);
    s->x = malloc(c * 4); s->y = malloc(c * 4); s->z = malloc(c * 4);
    s->mx = malloc(c * 4); s->my = malloc(c * 4); s->mz = malloc(c * 4);
    s->fx = malloc(c * 4); s->fy = malloc(c * 4); s->fz = malloc(c * 4);
    s->fsp = malloc(c); s->alive = malloc(c); s->busy = malloc(c);
    s->event = malloc(c * 4); s->key = malloc(c * 4); s->partner = malloc(c * 4);
    s->prop_b = malloc(c * 4); s->prop_r = malloc(c * 4); s->slot = malloc(c * 8);
    s->kids = malloc(c * sizeof(child_t));
    s->nxt = malloc(c * 4);
    if (!s->id || !s->sp || !s->x || !s->y || !s->z || !s->mx || !s->my || !s->mz || !s->fx ||
        !s->fy || !s->fz || !s->fsp || !s->alive || !s->busy || !s->event || !s->key ||
        !s->partner || !s->prop_b || !s->prop_r || !s->slot || !s->kids || !s->nxt) {
        orc_destroy(s);
        return NULL;
    }
    for (uint32_t i = 0; i < capacity; ++i) {
        s->key[i] = NONE32;
        s->event[i] = -1;
        s->partner[i] = NONE32;
    }
    if (bad) {
        orc_destroy(s);
        return NULL;
    }
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->id); free(s->sp); free(s->x); free(s->y); free(s->z);
    free(s->mx); free(s->my); free(s->mz); free(s->fx); free(s->fy); free(s->fz);
    free(s->fsp); free(s->alive); free(s->busy); free(s->event); free(s->key);
    free(s->partner); free(s->prop_b); free(s->prop_r); free(s->slot); free(s->kids);
    free(s->nxt); free(s->head);
    free(s);
}

const char* orc_last_error(const orc_sim* s) { return s ? s->err : "null sim"; }

int orc_add_species(orc_sim* s, float D, uint32_t count, int comp)
{
    if (s->failed) return ORC_E_STATE;
    if (s->tables_ready) return fail(s, ORC_E_STATE, "add_species after the model was finalized");
    if (s->ns >= MAXS) return fail(s, ORC_E_INVALID, "too many species");
    if (!(D >= 0.0f) || comp < 0 || comp >= s->ncomp)
        return fail(s, ORC_E_INVALID, "bad species parameters");
    s->D[s->ns] = D;
    s->init_count[s->ns] = count;
    s->init_comp[s->ns] = comp;
    return s->ns++;
}

int orc_add_rule(orc_sim* s, int kind, int r0, int r1, int p0, int p1, float radius,
                 double prob, int placement, float release, int from_comp, int to_comp)
{
    if (s->failed) return ORC_E_STATE;
    if (s->tables_ready) return fail(s, ORC_E_STATE, "add_rule after the model was finalized");
    if (s->nr >= MAXR) return fail(s, ORC_E_INVALID, "too many rules");
    int ns = s->ns;
#define SP_OK(v) ((v) >= 0 && (v) < ns)
#define PR_OK(v) ((v) == -1 || SP_OK(v))
    if (!(prob >= 0.0 && prob <= 1.0)) return fail(s, ORC_E_INVALID, "probability outside [0,1]");
    if (!SP_OK(r0) || !PR_OK(p0) || !PR_OK(p1)) return fail(s, ORC_E_INVALID, "unknown species");
    if (kind == ORC_BIMOL) {
        if (!SP_OK(r1)) return fail(s, ORC_E_INVALID, "unknown species");
        if (placement != ORC_KEEP) return fail(s, ORC_E_INVALID, "bimolecular rules keep positions");
        if (!(radius > 0.0f)) return fail(s, ORC_E_INVALID, "radius must be positive");
        for (int k = 0; k < s->nr; ++k) {
            const rule_t* o = &s->rule[k];
            if (o->kind == ORC_BIMOL &&
                ((o->r0 == r0 && o->r1 == r1) || (o->r0 == r1 && o->r1 == r0)))
                return fail(s, ORC_E_INVALID, "second bimolecular rule for one species pair");
        }
    } else if (kind == ORC_UNIMOL) {
        if (r1 != -1) return fail(s, ORC_E_INVALID, "unimolecular rule with two reactants");
        if (from_comp < -1 || from_comp >= s->ncomp)
            return fail(s, ORC_E_INVALID, "bad compartment");
        if (placement == ORC_KEEP) {
            if (p1 != -1) return fail(s, ORC_E_INVALID, "KEEP has one product");
        } else if (placement == ORC_SPLIT || placement == ORC_EMIT) {
            if (placement == ORC_SPLIT && p0 < 0) return fail(s, ORC_E_INVALID, "SPLIT needs two products");
            if (p1 < 0) return fail(s, ORC_E_INVALID, "missing emitted product");
            if (!(release >= 0.0f)) return fail(s, ORC_E_INVALID, "bad release radius");
        } else if (placement == ORC_TRANSLOCATE) {
            if (s->geometry != ORC_NESTED_SPHERES)
                return fail(s, ORC_E_INVALID, "translocation needs nested compartments");
            if (from_comp < 0 || to_comp < 0 || to_comp >= s->ncomp || to_comp == from_comp)
                return fail(s, ORC_E_INVALID, "bad translocation compartments");
            if (p1 != -1) return fail(s, ORC_E_INVALID, "TRANSLOCATE has one product");
            double rt = to_comp == 0 ? (double)s->Rin - (double)release
                                     : (double)s->Rin + (double)release;
            if (!(release >= 1e-3f) || !(rt > 0.0) || !(rt < (double)s->Rout))
                return fail(s, ORC_E_INVALID, "bad translocation offset");
        } else {
            return fail(s, ORC_E_INVALID, "bad placement");
        }
    } else {
        return fail(s, ORC_E_INVALID, "bad rule kind");
    }
#undef SP_OK
#undef PR_OK
    rule_t* r = &s->rule[s->nr];
    memset(r, 0, sizeof *r);
    r->kind = kind; r->r0 = r0; r->r1 = r1; r->p0 = p0; r->p1 = p1;
    r->placement = placement; r->from = from_comp; r->to = to_comp;
    r->radius = radius; r->prob = prob; r->release = release;
    return s->nr++;
}

int orc_set_search(orc_sim* s, int mode)
{
    if (mode != ORC_SEARCH_CELLS && mode != ORC_SEARCH_BRUTE)
        return fail(s, ORC_E_INVALID, "bad search mode");
    s->search = mode;
    return ORC_OK;
}

/* Per-species and per-rule constants, computed once in double and rounded
 * (sigma = sqrt(2 D dt) per axis; squared radii; Bernoulli thresholds
 * floor(p 2^32); cumulative unimolecular thresholds per species and
 * compartment in rule-id order), plus the consistency checks of Sec. 2
 * (referenced species exist, one event law per species). */
static uint64_t threshold(double p)
{
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

static int build_tables(orc_sim* s)
{
    if (s->tables_ready) return ORC_OK;
    if (s->ns == 0) return fail(s, ORC_E_INVALID, "no species");
    s->rmax = 0.0f;
    for (int k = 0; k < s->ns; ++k) {
        s->sigma[k] = (float)sqrt(2.0 * (double)s->D[k] * (double)s->dt);
        s->uni_n[k][0] = s->uni_n[k][1] = 0;
        s->is_claimer[k] = 0;
    }
    for (int r = 0; r < s->nr; ++r) {
        rule_t* ru = &s->rule[r];
        ru->r2 = (float)((double)ru->radius * (double)ru->radius);
        ru->release2 = (float)((double)ru->release * (double)ru->release);
        ru->thr = threshold(ru->prob);
        if (ru->placement == ORC_TRANSLOCATE)
            ru->target_r = (float)(ru->to == 0 ? (double)s->Rin - (double)ru->release
                                               : (double)s->Rin + (double)ru->release);
        if (ru->kind == ORC_BIMOL) {
            s->rule_of[ru->r0][ru->r1] = r;
            s->is_claimer[ru->r0] = 1;
            if (ru->radius > s->rmax) s->rmax = ru->radius;
        }
    }
    for (int k = 0; k < s->ns; ++k) {
        for (int c = 0; c < s->ncomp; ++c) {
            double cum = 0.0;
            for (int r = 0; r < s->nr; ++r) {
                const rule_t* ru = &s->rule[r];
                if (ru->kind != ORC_UNIMOL || ru->r0 != k) continue;
                if (ru->from != -1 && ru->from != c) continue;
                if (s->uni_n[k][c] >= MAXU)
                    return fail(s, ORC_E_INVALID, "too many unimolecular rules for one species");
                cum += ru->prob;
                if (cum > 1.0)
                    return fail(s, ORC_E_INVALID, "unimolecular probabilities of a species sum above 1");
                int j = s->uni_n[k][c]++;
                s->uni_rule[k][c][j] = r;
                s->uni_thr[k][c][j] = threshold(cum);
            }
        }
    }
    /* own search grid: cells no smaller than 1.1 R_max, at most 160 per axis */
    float extent = s->geometry == ORC_PERIODIC_BOX ? s->L : s->Rout * 2.0f;
    uint32_t og = 0;
    if (s->rmax > 0.0f) {
        double g = floor((double)extent / (1.1 * (double)s->rmax));
        og = g > 160.0 ? 160u : (uint32_t)g;
    }
    if (og < 3) og = 0; /* too coarse for a 27-cell stencil: brute force */
    s->og = og;
    if (og) {
        s->olo = s->geometry == ORC_PERIODIC_BOX ? 0.0f : -s->Rout;
        s->oinv = (float)((double)og / (double)extent);
        s->head = malloc((size_t)og * og * og * 4);
        if (!s->head) return fail(s, ORC_E_NOMEM, "out of memory");
    }
    s->tables_ready = 1;
    return ORC_OK;
}

/* O0: initial placement.  Agents get ids 0..N-1 in species order; agent i
 * tries Philox blocks (i, attempt, INIT, 0) for up to 64 attempts and keeps
 * the first uniform point of the bounding box of its compartment that lies
 * inside that compartment. */
static int place(orc_sim* s)
{
    uint64_t total = 0;
    for (int k = 0; k < s->ns; ++k) total += s->init_count[k];
    if (total > s->capacity) return fail(s, ORC_E_CAPACITY, "initial counts exceed capacity");
    uint32_t i = 0;
    for (int k = 0; k < s->ns; ++k) {
        int c = s->init_comp[k];
        for (uint32_t j = 0; j < s->init_count[k]; ++j, ++i) {
            int ok = 0;
            float x = 0, y = 0, z = 0;
            for (uint32_t a = 0; a < 64 && !ok; ++a) {
                uint32_t w[4];
                draw(s, i, a, PUR_INIT, 0, w);
                if (s->geometry == ORC_PERIODIC_BOX) {
                    x = wrap1(s, unif(w[0]) * s->L);
                    y = wrap1(s, unif(w[1]) * s->L);
                    z = wrap1(s, unif(w[2]) * s->L);
                    ok = 1;
                } else {
                    float R = (s->geometry == ORC_NESTED_SPHERES && c == 0) ? s->Rin : s->Rout;
                    x = (unif(w[0]) * 2.0f - 1.0f) * R;
                    y = (unif(w[1]) * 2.0f - 1.0f) * R;
                    z = (unif(w[2]) * 2.0f - 1.0f) * R;
                    float n2 = norm2(x, y, z);
                    if (s->geometry == ORC_SPHERE) ok = n2 <= s->Rout2;
                    else if (c == 0) ok = n2 < s->Rin2;
                    else ok = n2 >= s->Rin2 && n2 <= s->Rout2;
                }
            }
            if (!ok) return fail(s, ORC_E_DEVICE, "placement failed after 64 attempts");
            s->id[i] = i;
            s->sp[i] = (uint8_t)k;
            s->x[i] = x; s->y[i] = y; s->z[i] = z;
        }
    }
    s->n = i;
    s->next_id = i;
    s->t = 0;
    return ORC_OK;
}

static int finalize(orc_sim* s)
{
    if (s->failed) return ORC_E_STATE;
    int rc = build_tables(s);
    if (rc) { s->failed = 1; return rc; }
    if (!s->placed) {
        rc = place(s);
        if (rc) { s->failed = 1; return rc; }
        s->placed = 1;
    }
    return ORC_OK;
}

int orc_import(orc_sim* s, uint32_t n, const uint32_t* id, const uint8_t* sp, const float* x,
               const float* y, const float* z, uint32_t next_id, uint32_t t)
{
    if (s->failed) return ORC_E_STATE;
    int rc = build_tables(s);
    if (rc) { s->failed = 1; return rc; }
    if (n > s->capacity) return fail(s, ORC_E_CAPACITY, "import exceeds capacity");
    for (uint32_t i = 0; i < n; ++i) {
        if (sp[i] >= s->ns) return fail(s, ORC_E_INVALID, "unknown species in import");
        if (id[i] >= next_id) return fail(s, ORC_E_INVALID, "id not below next_id");
        if (!valid_at(s, x[i], y[i], z[i], comp_of(s, x[i], y[i], z[i])))
            return fail(s, ORC_E_INVALID, "imported position outside the volume");
        if (s->geometry == ORC_PERIODIC_BOX &&
            !(x[i] >= 0.0f && x[i] < s->L && y[i] >= 0.0f && y[i] < s->L && z[i] >= 0.0f && z[i] < s->L))
            return fail(s, ORC_E_INVALID, "imported position outside the box");
        s->id[i] = id[i]; s->sp[i] = sp[i];
        s->x[i] = x[i]; s->y[i] = y[i]; s->z[i] = z[i];
        s->key[i] = NONE32; s->event[i] = -1; s->partner[i] = NONE32;
    }
    s->n = n;
    s->next_id = next_id;
    s->t = t;
    s->placed = 1;
    return ORC_OK;
}

/* O8 helper: release offset u, uniform in the ball of radius delta, drawn
 * by cube rejection from Philox blocks (id, t, BIRTH, attempt), attempt <
 * 8; the offset is kept only if every placed product (p'+u, and p'-u for a
 * split) is inside the volume and in the parent's compartment.  No accepted
 * attempt: u = 0. */
static void release_offset(const orc_sim* s, const rule_t* ru, uint32_t id, float px, float py,
                           float pz, int both, float u[3])
{
    int c = comp_of(s, px, py, pz);
    for (uint32_t a = 0; a < 8; ++a) {
        uint32_t w[4];
        draw(s, id, s->t, PUR_BIRTH, a, w);
        float ux = (unif(w[0]) * 2.0f - 1.0f) * ru->release;
        float uy = (unif(w[1]) * 2.0f - 1.0f) * ru->release;
        float uz = (unif(w[2]) * 2.0f - 1.0f) * ru->release;
        if (!(norm2(ux, uy, uz) <= ru->release2)) continue;
        float ax = px + ux, ay = py + uy, az = pz + uz;
        if (s->geometry == ORC_PERIODIC_BOX) { ax = wrap1(s, ax); ay = wrap1(s, ay); az = wrap1(s, az); }
        if (!valid_at(s, ax, ay, az, c)) continue;
        if (both) {
            float bx = px - ux, by = py - uy, bz = pz - uz;
            if (s->geometry == ORC_PERIODIC_BOX) { bx = wrap1(s, bx); by = wrap1(s, by); bz = wrap1(s, bz); }
            if (!valid_at(s, bx, by, bz, c)) continue;
        }
        u[0] = ux; u[1] = uy; u[2] = uz;
        return;
    }
    u[0] = u[1] = u[2] = 0.0f;
}

static void add_child(orc_sim* s, uint32_t parent, int sp, float x, float y, float z)
{
    if (s->geometry == ORC_PERIODIC_BOX) { x = wrap1(s, x); y = wrap1(s, y); z = wrap1(s, z); }
    uint32_t slot;
#pragma omp atomic capture
    slot = s->nkids++;
    child_t* k = &s->kids[slot];
    k->parent = parent; k->sp = (uint8_t)sp; k->x = x; k->y = y; k->z = z;
}

/* O2..O5 and the unimolecular part of O8, for agent i. */
static void phase_move(orc_sim* s, uint32_t i)
{
    uint32_t id = s->id[i], t = s->t;
    int sp = s->sp[i];
    float x = s->x[i], y = s->y[i], z = s->z[i];
    int c0 = comp_of(s, x, y, z);

    uint32_t w[4];
    move_block(s->pkey, id, t, w);

    /* O2: one draw decides the unimolecular event (cumulative thresholds) */
    int ev = -1;
    uint32_t wu = event_word(w);
    for (int j = 0; j < s->uni_n[sp][c0]; ++j)
        if ((uint64_t)wu < s->uni_thr[sp][c0][j]) { ev = s->uni_rule[sp][c0][j]; break; }

    /* O3: Brownian move */
    float g[3];
    gauss3_w(w, g);
    float sg = s->sigma[sp];
    float x1 = fmaf(sg, g[0], x), y1 = fmaf(sg, g[1], y), z1 = fmaf(sg, g[2], z);

    /* O4: boundaries */
    if (s->geometry == ORC_PERIODIC_BOX) {
        x1 = wrap1(s, x1); y1 = wrap1(s, y1); z1 = wrap1(s, z1);
    } else {
        float n2 = norm2(x1, y1, z1);
        int reject = n2 > s->Rout2;
        if (s->geometry == ORC_NESTED_SPHERES && !reject && (n2 < s->Rin2 ? 0 : 1) != c0) reject = 1;
        if (reject) { x1 = x; y1 = y; z1 = z; }
    }
    s->mx[i] = x1; s->my[i] = y1; s->mz[i] = z1;
    s->key[i] = export_key(s, x1, y1, z1);  /* moved position; placement below may move it */
    s->event[i] = ev;
    s->partner[i] = NONE32;
    s->busy[i] = ev >= 0;
    s->alive[i] = 1;
    s->fsp[i] = (uint8_t)sp;
    s->fx[i] = x1; s->fy[i] = y1; s->fz[i] = z1;
    if (ev < 0) return;

    const rule_t* ru = &s->rule[ev];
    float u[3];
    switch (ru->placement) {
    case ORC_KEEP:
        if (ru->p0 < 0) s->alive[i] = 0;
        else s->fsp[i] = (uint8_t)ru->p0;
        break;
    case ORC_TRANSLOCATE: { /* O5: radial projection just across the membrane */
        float n2 = norm2(x1, y1, z1);
        if (n2 == 0.0f) {
            s->fx[i] = ru->target_r; s->fy[i] = 0.0f; s->fz[i] = 0.0f;
        } else {
            float f = ru->target_r / sqrtf(n2);
            s->fx[i] = x1 * f; s->fy[i] = y1 * f; s->fz[i] = z1 * f;
        }
        if (ru->p0 >= 0) s->fsp[i] = (uint8_t)ru->p0;
        s->key[i] = export_key(s, s->fx[i], s->fy[i], s->fz[i]);  /* O6: final position */
        break;
    }
    case ORC_SPLIT:
        release_offset(s, ru, id, x1, y1, z1, 1, u);
        s->fsp[i] = (uint8_t)ru->p0;
        s->fx[i] = x1 + u[0]; s->fy[i] = y1 + u[1]; s->fz[i] = z1 + u[2];
        if (s->geometry == ORC_PERIODIC_BOX) {
            s->fx[i] = wrap1(s, s->fx[i]); s->fy[i] = wrap1(s, s->fy[i]); s->fz[i] = wrap1(s, s->fz[i]);
        }
        add_child(s, id, ru->p1, x1 - u[0], y1 - u[1], z1 - u[2]);
        s->key[i] = export_key(s, s->fx[i], s->fy[i], s->fz[i]);  /* O6: final position */
        break;
    case ORC_EMIT:
        release_offset(s, ru, id, x1, y1, z1, 0, u);
        if (ru->p0 >= 0) s->fsp[i] = (uint8_t)ru->p0;
        add_child(s, id, ru->p1, x1 + u[0], y1 + u[1], z1 + u[2]);
        break;
    }
}

/* O7 helper: squared distance from a to b at the moved positions (minimum
 * image in the periodic box). */
static float dist2(const orc_sim* s, uint32_t a, uint32_t b)
{
    float dx = s->mx[b] - s->mx[a];
    float dy = s->my[b] - s->my[a];
    float dz = s->mz[b] - s->mz[a];
    if (s->geometry == ORC_PERIODIC_BOX) {
        if (dx > s->halfL) dx -= s->L; else if (dx < -s->halfL) dx += s->L;
        if (dy > s->halfL) dy -= s->L; else if (dy < -s->halfL) dy += s->L;
        if (dz > s->halfL) dz -= s->L; else if (dz < -s->halfL) dz += s->L;
    }
    return dx * dx + dy * dy + dz * dz;
}

/* O7: is b an eligible partner of claimer a, and under which rule */
static int consider(const orc_sim* s, uint32_t a, uint32_t b, int* best, float* best_d2,
                    int* best_r)
{
    if (b == a || s->busy[b]) return 0;
    int r = s->rule_of[s->sp[a]][s->sp[b]];
    if (r < 0) return 0;
    if (s->geometry == ORC_NESTED_SPHERES &&
        comp_of(s, s->mx[a], s->my[a], s->mz[a]) != comp_of(s, s->mx[b], s->my[b], s->mz[b]))
        return 0;
    float d2 = dist2(s, a, b);
    if (!(d2 <= s->rule[r].r2)) return 0;
    if (*best < 0 || d2 < *best_d2 || (d2 == *best_d2 && s->id[b] < s->id[*best])) {
        *best = (int)b; *best_d2 = d2; *best_r = r;
    }
    return 1;
}

static uint32_t ocell(const orc_sim* s, float v) { return cell_axis(v, s->olo, s->oinv, s->og); }

static void build_cells(orc_sim* s)
{
    uint32_t g = s->og;
    size_t nc = (size_t)g * g * g;
    for (size_t c = 0; c < nc; ++c) s->head[c] = -1;
    for (uint32_t i = 0; i < s->n; ++i) {
        if (s->busy[i]) continue;
        uint32_t c = ocell(s, s->mx[i]) + g * (ocell(s, s->my[i]) + g * ocell(s, s->mz[i]));
        s->nxt[i] = s->head[c];
        s->head[c] = (int32_t)i;
    }
}

/* O6/O7: argmin over eligible partners of (d^2, id), by the cell list. */
static int search_cells(const orc_sim* s, uint32_t a, int* best_r)
{
    int g = (int)s->og, best = -1;
    float bd = 0.0f;
    int cx = (int)ocell(s, s->mx[a]), cy = (int)ocell(s, s->my[a]), cz = (int)ocell(s, s->mz[a]);
    int periodic = s->geometry == ORC_PERIODIC_BOX;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int x = cx + dx, y = cy + dy, z = cz + dz;
                if (periodic) {
                    x = (x + g) % g; y = (y + g) % g; z = (z + g) % g;
                } else if (x < 0 || y < 0 || z < 0 || x >= g || y >= g || z >= g) {
                    continue;
                }
                for (int b = s->head[x + g * (y + g * z)]; b >= 0; b = s->nxt[b])
                    consider(s, a, (uint32_t)b, &best, &bd, best_r);
            }
    return best;
}

static int search_brute(const orc_sim* s, uint32_t a, int* best_r)
{
    int best = -1;
    float bd = 0.0f;
    for (uint32_t b = 0; b < s->n; ++b) consider(s, a, b, &best, &bd, best_r);
    return best;
}

static uint32_t prio_of(const orc_sim* s, uint32_t ida, uint32_t idb)
{
    uint32_t lo = ida < idb ? ida : idb, hi = ida < idb ? idb : ida, w[4];
    draw(s, lo, s->t, PUR_PRIO, hi, w);
    return w[0];
}

static int cmp_child(const void* a, const void* b)
{
    uint32_t x = ((const child_t*)a)->parent, y = ((const child_t*)b)->parent;
    return x < y ? -1 : x > y;
}

/* One step: O2..O10 in order. */
static int step_one(orc_sim* s)
{
    uint32_t n = s->n;
    s->nkids = 0;
#pragma omp parallel for schedule(static)
    for (uint32_t i = 0; i < n; ++i) phase_move(s, i);

    /* O6/O7: proposals */
    int use_cells = s->search == ORC_SEARCH_CELLS && s->og;
    if (use_cells) build_cells(s);
    for (uint32_t a = 0; a < n; ++a) {
        s->prop_b[a] = -1;
        s->slot[a] = UINT64_MAX;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (uint32_t a = 0; a < n; ++a) {
        if (s->busy[a] || !s->is_claimer[s->sp[a]]) continue;
        int r = -1;
        int b = use_cells ? search_cells(s, a, &r) : search_brute(s, a, &r);
        if (b < 0) continue;
        uint32_t w[4];
        draw(s, s->id[a], s->t, PUR_PAIR, 0, w);
        if ((uint64_t)w[0] < s->rule[r].thr) {
            s->prop_b[a] = b;
            s->prop_r[a] = r;
        }
    }
    /* O7: claim slots keep the smallest (prio, other id) key */
    for (uint32_t a = 0; a < n; ++a) {
        int b = s->prop_b[a];
        if (b < 0) continue;
        uint64_t pr = (uint64_t)prio_of(s, s->id[a], s->id[b]) << 32;
        uint64_t ka = pr | s->id[b], kb = pr | s->id[a];
        if (ka < s->slot[a]) s->slot[a] = ka;
        if (kb < s->slot[b]) s->slot[b] = kb;
    }
    /* O7/O8: confirmed pairs fire; mutual proposals fire once, the lower id
     * taking the claimer's role */
    for (uint32_t a = 0; a < n; ++a) {
        int b = s->prop_b[a];
        if (b < 0) continue;
        uint64_t pr = (uint64_t)prio_of(s, s->id[a], s->id[b]) << 32;
        if (s->slot[a] != (pr | s->id[b]) || s->slot[b] != (pr | s->id[a])) continue;
        if (s->prop_b[b] == (int)a && s->id[b] < s->id[a]) continue;
        const rule_t* ru = &s->rule[s->prop_r[a]];
        if (ru->p0 < 0) s->alive[a] = 0; else s->fsp[a] = (uint8_t)ru->p0;
        if (ru->p1 < 0) s->alive[b] = 0; else s->fsp[b] = (uint8_t)ru->p1;
        s->partner[a] = s->id[b];
        s->partner[b] = s->id[a];
    }

    /* O9: compaction of survivors, children appended in parent-id order */
    uint32_t m = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!s->alive[i]) continue;
        s->id[m] = s->id[i];
        s->sp[m] = s->fsp[i];
        s->x[m] = s->fx[i]; s->y[m] = s->fy[i]; s->z[m] = s->fz[i];
        s->key[m] = s->key[i]; s->event[m] = s->event[i]; s->partner[m] = s->partner[i];
        ++m;
    }
    if ((uint64_t)m + s->nkids > s->capacity) {
        s->failed = 1;
        return fail(s, ORC_E_CAPACITY, "agent capacity exceeded by births");
    }
    qsort(s->kids, s->nkids, sizeof(child_t), cmp_child);
    for (uint32_t k = 0; k < s->nkids; ++k, ++m) {
        s->id[m] = s->next_id++;
        s->sp[m] = s->kids[k].sp;
        s->x[m] = s->kids[k].x; s->y[m] = s->kids[k].y; s->z[m] = s->kids[k].z;
        s->key[m] = NONE32; s->event[m] = -1; s->partner[m] = NONE32;
    }
    s->n = m;
    s->t += 1; /* O10 */
    return ORC_OK;
}

int orc_step(orc_sim* s, uint32_t n_steps)
{
    int rc = finalize(s);
    if (rc) return rc;
    for (uint32_t k = 0; k < n_steps; ++k) {
        rc = step_one(s);
        if (rc) return rc;
    }
    return ORC_OK;
}

int orc_counts(orc_sim* s, uint64_t* out, uint32_t n_species, uint64_t* out_step)
{
    int rc = finalize(s);
    if (rc) return rc;
    for (uint32_t k = 0; k < n_species; ++k) out[k] = 0;
    for (uint32_t i = 0; i < s->n; ++i)
        if (s->sp[i] < n_species) out[s->sp[i]] += 1;
    if (out_step) *out_step = s->t;
    return ORC_OK;
}

int orc_size(orc_sim* s, uint32_t* n, uint32_t* next_id)
{
    int rc = finalize(s);
    if (rc) return rc;
    *n = s->n;
    if (next_id) *next_id = s->next_id;
    return ORC_OK;
}

static const orc_sim* g_sort_sim;
static int cmp_idx(const void* a, const void* b)
{
    uint32_t x = g_sort_sim->id[*(const uint32_t*)a], y = g_sort_sim->id[*(const uint32_t*)b];
    return x < y ? -1 : x > y;
}

int orc_export(orc_sim* s, uint32_t cap, uint32_t* id, uint8_t* sp, float* x, float* y, float* z,
               uint32_t* key, int32_t* event, uint32_t* partner)
{
    int rc = finalize(s);
    if (rc) return rc;
    if (cap < s->n) return fail(s, ORC_E_INVALID, "export buffer too small");
    uint32_t* idx = malloc((size_t)(s->n ? s->n : 1) * 4);
    if (!idx) return fail(s, ORC_E_NOMEM, "out of memory");
    for (uint32_t i = 0; i < s->n; ++i) idx[i] = i;
    g_sort_sim = s;
    qsort(idx, s->n, 4, cmp_idx);
    for (uint32_t k = 0; k < s->n; ++k) {
        uint32_t i = idx[k];
        if (id) id[k] = s->id[i];
        if (sp) sp[k] = s->sp[i];
        if (x) x[k] = s->x[i];
        if (y) y[k] = s->y[i];
        if (z) z[k] = s->z[i];
        if (key) key[k] = s->key[i];
        if (event) event[k] = s->event[i];
        if (partner) partner[k] = s->partner[i];
    }
    free(idx);
    return ORC_OK;
}

/* Threads of the two parallel loops (0: OpenMP's default); returns the
 * number the next step will use. */
int orc_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
