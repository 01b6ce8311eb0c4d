/*
 * CPU oracle of the SVT linearized track fitter.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or loads this file;
 * only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no header, helper or table with the HIP implementation.
 *
 * What it computes (Gianelle et al., "Applications of Many-Core Technologies to On-line Event
 * Reconstruction in High Energy Physics Experiments", IEEE NSS 2013):
 *   - Section II: a fit on every combination of hits inside a road, each track parameter being
 *     a scalar product of pre-defined constants with the hits plus an offset (the one equation
 *     of the paper, p_i = f_i . x_i + q_i), done with table lookups and integer add/multiply.
 *   - Section II-A: the serial code is three functions -- unpack the input and fill the data
 *     structures, compute all combinations of hits of each road, fit each combination -- run
 *     inside three nested loops over events, roads and combinations.  This file keeps exactly
 *     that structure, one plain loop per stage, with no blocking or reordering.
 *
 * Readings where the paper is silent (word format, constant sizes, shift, chi-square rule) are
 * listed at each function and collected in the design notes of the repository:
 *   R1  word bits, LSB first: coord 13 | layer 3 | road tag 8 | event tag 8
 *   R2  coord is a two's-complement 13-bit integer (-4096 .. 4095)
 *   R3  a layer field >= n_layers is an input error, reported at the smallest word index
 *   R4  tags are delimiters: a new event starts where the event tag changes, a new road where
 *       either tag changes; events and roads are numbered by order of appearance
 *   R5  the constant set of a road is selected by its 8-bit road tag
 *   R6  hits of a road are grouped by layer, keeping stream order inside a layer; more than
 *       max_hits hits in one layer is an input error reported at the smallest road index;
 *       a road tag with no constant set (tag >= n_sets) is an input error, reported after
 *       the hit-count errors, at the smallest road index
 *   R7  combination k of a road is a mixed-radix number with layer 0 most significant (the
 *       nested loops "for h0 .. for h4")
 *   R8  the offset is added before the shift: v_j = floor((sum_l f_jl x_l + q_j) / 2^shift)
 *   R9  the shift rounds toward minus infinity (arithmetic shift of the exact integer)
 *   R10 rows 0-2 are the track parameters, rows 3-5 chi-square components;
 *       chi2 = c0^2 + c1^2 + c2^2 computed exactly in 64 bits
 *   R11 a combination is kept when chi2 <= cut
 *   R12 the best track of a road is its kept combination of smallest chi2, the first one in
 *       enumeration order among equal chi2 (what a serial loop with a strict "<" keeps)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_ERR_ARG (-1)
#define ORA_ERR_LAYER (-2)
#define ORA_ERR_HITS (-3)
#define ORA_ERR_SET (-6)

#define ORA_MAX_LAYERS 5
#define ORA_MAX_HITS 8

typedef struct {
    int32_t n_layers;
    int32_t shift;
    int64_t chi2_cut;
    int32_t max_hits;
    int32_t n_sets;
} ora_config;

/* Output buffers, all host memory, sized by ora_count(). Any pointer may be NULL to skip it. */
typedef struct {
    /* road table, [n_roads] */
    int32_t *road_event;
    int32_t *road_set;
    int64_t *road_hit_begin;
    uint32_t *road_nhits;      /* 4 bits per layer, layer l in bits 4l..4l+3 */
    int64_t *road_combo_begin;
    int32_t *road_ncombo;
    /* hit coordinates grouped by layer inside each road, [n_words] */
    int16_t *hit_coord;
    /* per combination, [n_combos] */
    int32_t *combo_road;
    uint32_t *combo_hits;      /* hit index inside its layer, 4 bits per layer */
    int32_t *p0, *p1, *p2;
    int32_t *c0, *c1, *c2;
    int64_t *chi2;
    uint8_t *accept;
    /* best track per road, [n_roads] */
    int32_t *best_nacc;
    int32_t *best_k;
    int32_t *best_p0, *best_p1, *best_p2;
    int64_t *best_chi2;
    /* ascending indices of kept combinations, [n_combos] */
    int64_t *kept;
} ora_out;

/* ---- one decoded hit word (R1, R2) ------------------------------------------------------ */
typedef struct {
    int32_t coord;
    int32_t layer;
    int32_t rtag;
    int32_t etag;
} ora_hit;

static ora_hit decode_word(uint32_t w)
{
    ora_hit h;
    int32_t raw = (int32_t)(w & 0x1FFFu);
    h.coord = (raw >= 4096) ? raw - 8192 : raw; /* two's complement of 13 bits */
    h.layer = (int32_t)((w >> 13) & 0x7u);
    h.rtag = (int32_t)((w >> 16) & 0xFFu);
    h.etag = (int32_t)((w >> 24) & 0xFFu);
    return h;
}

/* floor(a / 2^s) for any sign of a, written without relying on the shift of negatives (R9) */
static int64_t floor_div_pow2(int64_t a, int32_t s)
{
    int64_t d = (int64_t)1 << s;
    int64_t q = a / d;      /* C division truncates toward zero */
    if ((a % d) != 0 && a < 0)
        q -= 1;
    return q;
}

/* ---- unpack: decode and cut the stream into events and roads (section II-A; R3, R4) ------ */
typedef struct {
    int64_t begin; /* first word */
    int64_t len;   /* number of words */
    int32_t event; /* event ordinal */
    int32_t rtag;
} ora_road;

/* Returns ORA_OK or ORA_ERR_LAYER with *err_index = smallest bad word.  Fills roads[] when
 * non-NULL; always sets *n_roads and *n_events. */
static int32_t segment_stream(const uint32_t *words, int64_t n_words, int32_t n_layers,
                              ora_road *roads, int64_t *n_roads, int64_t *n_events,
                              int64_t *err_index)
{
    int64_t nr = 0, ne = 0;
    ora_hit prev = {0, 0, -1, -1};
    for (int64_t i = 0; i < n_words; i++) {
        ora_hit h = decode_word(words[i]);
        if (h.layer >= n_layers) {
            *err_index = i;
            *n_roads = 0;
            *n_events = 0;
            return ORA_ERR_LAYER;
        }
        int new_event = (i == 0) || (h.etag != prev.etag);
        int new_road = new_event || (h.rtag != prev.rtag);
        if (new_event)
            ne++;
        if (new_road) {
            if (roads) {
                roads[nr].begin = i;
                roads[nr].len = 0;
                roads[nr].event = (int32_t)(ne - 1);
                roads[nr].rtag = h.rtag;
            }
            nr++;
        }
        if (roads)
            roads[nr - 1].len++;
        prev = h;
    }
    *n_roads = nr;
    *n_events = ne;
    return ORA_OK;
}

/* ---- unpack: group one road's hits by layer, stable (R6) -------------------------------- */
typedef struct {
    int32_t n[ORA_MAX_LAYERS];                   /* hits per layer */
    int32_t x[ORA_MAX_LAYERS][ORA_MAX_HITS];     /* coordinates, stream order inside a layer */
} ora_grouped;

/* Returns 0 when every layer holds at most max_hits hits, -1 otherwise. */
static int group_road(const uint32_t *words, const ora_road *rd, int32_t n_layers,
                      int32_t max_hits, ora_grouped *g)
{
    memset(g, 0, sizeof(*g));
    for (int64_t i = rd->begin; i < rd->begin + rd->len; i++) {
        ora_hit h = decode_word(words[i]);
        if (g->n[h.layer] >= max_hits)
            return -1;
        g->x[h.layer][g->n[h.layer]] = h.coord;
        g->n[h.layer]++;
    }
    (void)n_layers;
    return 0;
}

/* ---- combine: number of one-hit-per-layer combinations of a road (section II-A) ---------- */
static int64_t road_combinations(const ora_grouped *g, int32_t n_layers)
{
    int64_t c = 1;
    for (int l = 0; l < n_layers; l++)
        c *= g->n[l];
    return c;
}

/* ---- fit: the linearized fit of one combination (section II, the scalar-product equation;
 *      R5, R8, R9, R10) ------------------------------------------------------------------- */
typedef struct {
    int32_t v[6];
    int64_t chi2;
} ora_fit;

static ora_fit fit_one(const int16_t *f_set /* [6][5] */, const int32_t *q_set /* [6] */,
                       const int32_t *x /* [5] */, int32_t n_layers, int32_t shift)
{
    ora_fit r;
    for (int j = 0; j < 6; j++) {
        int64_t a = 0;
        for (int l = 0; l < n_layers; l++)
            a += (int64_t)f_set[j * 5 + l] * (int64_t)x[l];
        a += (int64_t)q_set[j];
        r.v[j] = (int32_t)floor_div_pow2(a, shift);
    }
    r.chi2 = 0;
    for (int j = 3; j < 6; j++)
        r.chi2 += (int64_t)r.v[j] * (int64_t)r.v[j];
    return r;
}

static int config_ok(const ora_config *cfg)
{
    return cfg && cfg->n_layers == ORA_MAX_LAYERS && cfg->shift >= 1 && cfg->shift <= 30 &&
           cfg->max_hits >= 1 && cfg->max_hits <= ORA_MAX_HITS && cfg->n_sets >= 1 &&
           cfg->n_sets <= 256;
}

/* Sizes of the outputs.  Also reports input errors exactly as ora_run does. */
int32_t ora_count(const uint32_t *words, int64_t n_words, const ora_config *cfg,
                  int64_t *n_roads, int64_t *n_events, int64_t *n_combos, int64_t *err_index)
{
    if (!config_ok(cfg) || n_words < 0 || (n_words > 0 && !words))
        return ORA_ERR_ARG;
    *err_index = -1;
    *n_combos = 0;
    int32_t st = segment_stream(words, n_words, cfg->n_layers, NULL, n_roads, n_events, err_index);
    if (st != ORA_OK)
        return st;
    ora_road *roads = (ora_road *)malloc(sizeof(ora_road) * (size_t)(*n_roads > 0 ? *n_roads : 1));
    segment_stream(words, n_words, cfg->n_layers, roads, n_roads, n_events, err_index);
    int64_t total = 0;
    for (int64_t r = 0; r < *n_roads; r++) {
        ora_grouped g;
        if (group_road(words, &roads[r], cfg->n_layers, cfg->max_hits, &g) != 0) {
            *err_index = r;
            free(roads);
            return ORA_ERR_HITS;
        }
        total += road_combinations(&g, cfg->n_layers);
    }
    for (int64_t r = 0; r < *n_roads; r++) {
        if (roads[r].rtag >= cfg->n_sets) {
            *err_index = r;
            free(roads);
            return ORA_ERR_SET;
        }
    }
    *n_combos = total;
    free(roads);
    return ORA_OK;
}

/* The whole path: unpack, combine, fit, select, in the loop nest events -> roads ->
 * combinations of section II-A.  The combination loop runs h0 outermost .. h4 innermost (R7). */
int32_t ora_run(const uint32_t *words, int64_t n_words, const int16_t *f, const int32_t *q,
                const ora_config *cfg, const ora_out *out, int64_t *n_kept, int64_t *err_index)
{
    int64_t n_roads, n_events, n_combos;
    int32_t st = ora_count(words, n_words, cfg, &n_roads, &n_events, &n_combos, err_index);
    if (st != ORA_OK)
        return st;
    if (!f || !q || !out)
        return ORA_ERR_ARG;

    ora_road *roads = (ora_road *)malloc(sizeof(ora_road) * (size_t)(n_roads > 0 ? n_roads : 1));
    segment_stream(words, n_words, cfg->n_layers, roads, &n_roads, &n_events, err_index);

    const int L = cfg->n_layers;
    int64_t combo = 0; /* global combination index */
    int64_t nk = 0;
    int64_t r = 0;
    for (int64_t ev = 0; ev < n_events; ev++) {                 /* loop on events */
        for (; r < n_roads && roads[r].event == ev; r++) {      /* loop on roads */
            const ora_road *rd = &roads[r];
            ora_grouped g;
            group_road(words, rd, L, cfg->max_hits, &g); /* checked in ora_count */
            int64_t nc = road_combinations(&g, L);
            int32_t s = rd->rtag;
            const int16_t *fs = f + (size_t)s * 30;
            const int32_t *qs = q + (size_t)s * 6;

            uint32_t packed_n = 0;
            for (int l = 0; l < L; l++)
                packed_n |= (uint32_t)g.n[l] << (4 * l);
            if (out->road_event) out->road_event[r] = rd->event;
            if (out->road_set) out->road_set[r] = s;
            if (out->road_hit_begin) out->road_hit_begin[r] = rd->begin;
            if (out->road_nhits) out->road_nhits[r] = packed_n;
            if (out->road_combo_begin) out->road_combo_begin[r] = combo;
            if (out->road_ncombo) out->road_ncombo[r] = (int32_t)nc;
            if (out->hit_coord) {
                int64_t o = rd->begin;
                for (int l = 0; l < L; l++)
                    for (int h = 0; h < g.n[l]; h++)
                        out->hit_coord[o++] = (int16_t)g.x[l][h];
            }

            int32_t best_k = -1, best_v[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
            int64_t best_chi2 = INT64_MAX;
            int32_t nacc = 0;
            int32_t k = 0;
            /* loop on combinations: one hit per layer, layer 0 most significant */
            for (int h0 = 0; h0 < g.n[0]; h0++)
            for (int h1 = 0; h1 < g.n[1]; h1++)
            for (int h2 = 0; h2 < g.n[2]; h2++)
            for (int h3 = 0; h3 < g.n[3]; h3++)
            for (int h4 = 0; h4 < g.n[4]; h4++) {
                int32_t x[5] = {g.x[0][h0], g.x[1][h1], g.x[2][h2], g.x[3][h3], g.x[4][h4]};
                ora_fit ft = fit_one(fs, qs, x, L, cfg->shift);
                int acc = ft.chi2 <= cfg->chi2_cut;                        /* R11 */
                if (out->combo_road) out->combo_road[combo] = (int32_t)r;
                if (out->combo_hits)
                    out->combo_hits[combo] = (uint32_t)h0 | ((uint32_t)h1 << 4) |
                                             ((uint32_t)h2 << 8) | ((uint32_t)h3 << 12) |
                                             ((uint32_t)h4 << 16);
                if (out->p0) out->p0[combo] = ft.v[0];
                if (out->p1) out->p1[combo] = ft.v[1];
                if (out->p2) out->p2[combo] = ft.v[2];
                if (out->c0) out->c0[combo] = ft.v[3];
                if (out->c1) out->c1[combo] = ft.v[4];
                if (out->c2) out->c2[combo] = ft.v[5];
                if (out->chi2) out->chi2[combo] = ft.chi2;
                if (out->accept) out->accept[combo] = (uint8_t)acc;
                if (acc) {
                    nacc++;
                    if (ft.chi2 < best_chi2) {                              /* R12 */
                        best_chi2 = ft.chi2;
                        best_k = k;
                        best_v[0] = ft.v[0];
                        best_v[1] = ft.v[1];
                        best_v[2] = ft.v[2];
                    }
                    if (out->kept) out->kept[nk] = combo;
                    nk++;
                }
                combo++;
                k++;
            }
            if (out->best_nacc) out->best_nacc[r] = nacc;
            if (out->best_k) out->best_k[r] = best_k;
            if (out->best_p0) out->best_p0[r] = best_v[0];
            if (out->best_p1) out->best_p1[r] = best_v[1];
            if (out->best_p2) out->best_p2[r] = best_v[2];
            if (out->best_chi2) out->best_chi2[r] = best_chi2;
        }
    }
    free(roads);
    *n_kept = nk;
    *err_index = -1;
    return ORA_OK;
}
