/*
 * pyro_oracle.c -- CPU oracle for one Swendsen-Wang sweep of the ferromagnetic
 * O(n) model (n = 1 Ising, 2 XY, 3 Heisenberg) on the periodic pyrochlore
 * lattice, following Soldatov, Nefedev, Komura, Okabe, "Large-scale
 * calculation of ferromagnetic spin systems on the pyrochlore lattice".
 *
 * THIS IS TEST INFRASTRUCTURE.  It is a plain, slow, single-threaded,
 * obviously-correct restatement of the method, used only by the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark.  The product
 * (the HIP library) never links, loads or calls it, and it shares no code,
 * header, table or constant generator with the product.
 *
 * What it computes, and where each piece comes from:
 *   - Lattice: 16-site cubic unit cell, L x L x L cells, periodic
 *     (Sec. 2).  Sites are placed by geometry (FCC points plus a
 *     four-site tetrahedral basis) and the tetrahedra are found by looking
 *     positions up; no closed-form neighbour arithmetic is used here.
 *   - Hamiltonian H = -J sum_<ij> s_i . s_j, unit n-vectors (Sec. 2, Eq. 1).
 *   - Swendsen-Wang multi-cluster update with Wolff's embedding for n > 1
 *     (Sec. 1 and Sec. 2): activate each bond with probability
 *     1 - exp(-2 beta J s_i s_j) when the (projected) spins are parallel,
 *     label the connected clusters (breadth-first search, label = smallest
 *     site index in the cluster), flip (reflect) each cluster with
 *     probability 1/2.
 *   - Measurement: M, m = M/N, m^2, m^4 per sweep (Sec. 3.1, Eq. 2) and the
 *     energy E = H (Eq. 1).
 *   - Site dilution (the extension named in Sec. 4): a vacant site is a
 *     zero spin (Ising 0, O(n) the zero vector).  It carries no bond (for
 *     O(n) the projected product is 0, so the bond never activates), stays
 *     its own one-site cluster and stays zero under flips; m is M/N with N
 *     all sites, vacant or not.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     counter = (unit, sweep, stream, attempt), key = seed.  The paper does
 *     not name its generator; the counter layout is this project's reading.
 *
 * Every function below is written for clarity, not speed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ISING 1
#define ORC_XY 2
#define ORC_HEIS 3

#define ORC_KIND_PYRO 0
#define ORC_KIND_SC 1
#define ORC_KIND_EDGES 2

/* Random-number streams (third counter word). */
#define ST_BOND 0u
#define ST_FLIP 1u
#define ST_INIT 2u
#define ST_AXIS 3u
#define ST_BOND_LO 4u

/* Deliberate mistakes that tests plant to show the pins catch them. */
#define PLANT_NONE 0
#define PLANT_HALF_BETA 1   /* use 1 - exp(-beta J) instead of 1 - exp(-2 beta J) */
#define PLANT_FLIP_ALL 2    /* flip every cluster instead of each with prob. 1/2 */
#define PLANT_DROP_BONDS 3  /* bonds with odd index never activate */
#define PLANT_REFLECT_SIGN 4 /* O(n): s + 2 (s.r) r instead of s - 2 (s.r) r */
#define PLANT_ANTI 5        /* Ising: activate antiparallel instead of parallel */
#define PLANT_VACANT_JOIN 6 /* Ising: let two vacant sites activate their bond */

typedef struct {
    int64_t sweep;    /* global 0-based index of the sweep this record follows */
    int64_t bond_sum; /* Ising: sum over bonds of s_i s_j (exact) */
    int64_t M_int;    /* Ising: sum of s_i (exact) */
    int64_t pad;
    double E;         /* -J sum_<ij> s_i . s_j */
    double M[3];      /* sum_i s_i, per component */
    double m2, m4;    /* m = |M|/N, m2 = m*m, m4 = m2*m2 */
} orc_record;

typedef struct orc {
    int kind, L, model, n, start, plant;
    int64_t N, NB;
    int32_t *ba, *bb;        /* endpoints of bond b: ba[b] < tetra order < bb[b] */
    int64_t *adj_off;        /* CSR: bonds incident to each site */
    int64_t *adj_bond;
    double T, J;
    uint64_t seed;
    uint64_t thr;            /* Ising: activation threshold on a 32-bit uniform */
    float x0;                /* O(n): (float)(2 beta J) */
    int8_t *s8;              /* Ising spins, +1 / -1 */
    float *sv;               /* O(n) spins, site-major [N][n] */
    float *sigma;            /* O(n) projections of the current sweep */
    uint8_t *active;         /* activation of each bond, last sweep */
    int32_t *label;          /* cluster label of each site, last sweep */
    int32_t *queue;
    uint8_t *flip;
    int64_t t;               /* global sweep counter */
} orc;

/* ------------------------------------------------------------------------ */
/* Philox4x32 with 10 rounds, from the description in Salmon et al. (2011):  */
/* each round multiplies words 0 and 2 by two fixed odd constants, swaps the */
/* halves crosswise with the odd words and the round key, and the two key    */
/* words advance by two Weyl constants between rounds.                       */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint64_t c0, int64_t t, uint32_t stream,
                 uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)c0, (uint32_t)t, stream, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* Ising bond uniform r32(b): top byte from byte (b mod 16) of the BOND call
 * for b/16, low 24 bits from word (b mod 4) of the BOND_LO call for b/4. */
static uint32_t ising_bond_uniform(uint64_t seed, uint64_t b, int64_t t)
{
    uint32_t w[4], v[4];
    draw(seed, b >> 4, t, ST_BOND, 0, w);
    uint32_t k = (uint32_t)(b & 15);
    uint32_t hi8 = (w[k >> 2] >> (8 * (k & 3))) & 0xFFu;
    draw(seed, b >> 2, t, ST_BOND_LO, 0, v);
    uint32_t lo24 = v[b & 3] & 0xFFFFFFu;
    return (hi8 << 24) | lo24;
}

/* O(n) bond uniform: word (b mod 4) of the BOND call for b/4. */
static uint32_t on_bond_uniform(uint64_t seed, uint64_t b, int64_t t)
{
    uint32_t w[4];
    draw(seed, b >> 2, t, ST_BOND, 0, w);
    return w[b & 3];
}

/* Flip coin of the cluster whose label (smallest site index) is r. */
static int flip_bit(uint64_t seed, uint64_t r, int64_t t)
{
    uint32_t w[4];
    draw(seed, r >> 7, t, ST_FLIP, 0, w);
    return (int)((w[(r >> 5) & 3] >> (r & 31)) & 1u);
}

/* Uniform unit n-vector (n = 2, 3) by rejection from the cube [-1,1]^n.
 * Attempt a uses counter (c0, t, stream, a); at most 64 attempts, then the
 * x unit vector (probability below 1e-17). */
static void unit_vector(uint64_t seed, uint64_t c0, int64_t t, uint32_t stream,
                        int n, float v_out[3])
{
    for (uint32_t a = 0; a < 64; ++a) {
        uint32_t w[4];
        draw(seed, c0, t, stream, a, w);
        float v[3];
        for (int k = 0; k < 3; ++k)
            v[k] = (float)(int32_t)w[k] * 0x1p-31f;
        float r2 = v[0] * v[0];
        r2 = fmaf(v[1], v[1], r2);
        if (n == 3) r2 = fmaf(v[2], v[2], r2);
        if (r2 > 1e-12f && r2 <= 1.0f) {
            float nr = sqrtf(r2);
            v_out[0] = v[0] / nr;
            v_out[1] = v[1] / nr;
            v_out[2] = (n == 3) ? v[2] / nr : 0.0f;
            return;
        }
    }
    v_out[0] = 1.0f; v_out[1] = 0.0f; v_out[2] = 0.0f;
}

void orc_axis(uint64_t seed, int64_t t, int n, float r[3])
{
    unit_vector(seed, 0, t, ST_AXIS, n, r);
}

/* Activation threshold for the Ising model: bond is active when the 32-bit
 * uniform is below floor(p * 2^32), p = 1 - exp(-2 J / T). */
uint64_t orc_ising_threshold(double T, double J)
{
    double p = -expm1(-2.0 * J / T);
    return (uint64_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------ */
/* Lattices                                                                  */
/* ------------------------------------------------------------------------ */

/* Pyrochlore geometry in units of a/4 (a = cubic cell edge).  The cubic cell
 * holds four FCC points F_f; each carries a tetrahedron of four sites at
 * offsets B_mu.  Site (cell, f, mu) has index 16*cell + 4*f + mu. */
static const int FCC[4][3] = {{0, 0, 0}, {0, 2, 2}, {2, 0, 2}, {2, 2, 0}};
static const int BAS[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
static const int PAIR[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

static int64_t wrap(int64_t v, int64_t m) { v %= m; return v < 0 ? v + m : v; }

/* Site index at a lattice position (any integer vector; wrapped), -1 if the
 * position holds no site. */
static int64_t pyro_site_at(int L, const int64_t p_in[3])
{
    int64_t p[3], c[3], o[3];
    for (int k = 0; k < 3; ++k) {
        p[k] = wrap(p_in[k], 4 * (int64_t)L);
        c[k] = p[k] / 4;
        o[k] = p[k] - 4 * c[k];
    }
    for (int f = 0; f < 4; ++f)
        for (int mu = 0; mu < 4; ++mu)
            if (FCC[f][0] + BAS[mu][0] == o[0] && FCC[f][1] + BAS[mu][1] == o[1] &&
                FCC[f][2] + BAS[mu][2] == o[2]) {
                int64_t cell = (c[2] * L + c[1]) * L + c[0];
                return 16 * cell + 4 * f + mu;
            }
    return -1;
}

void orc_pyro_position(int L, int64_t i, int32_t pos[3])
{
    int64_t cell = i / 16, f = (i / 4) % 4, mu = i % 4;
    int64_t x = cell % L, y = (cell / L) % L, z = cell / ((int64_t)L * L);
    pos[0] = (int32_t)(4 * x + FCC[f][0] + BAS[mu][0]);
    pos[1] = (int32_t)(4 * y + FCC[f][1] + BAS[mu][1]);
    pos[2] = (int32_t)(4 * z + FCC[f][2] + BAS[mu][2]);
}

/* Bond list: cell c owns 8 tetrahedra, t = f for the up tetrahedron
 * {R + B_mu} and t = 4 + f for the down tetrahedron {R - B_mu} around the
 * FCC point R = 4c + F_f; bond b = 48*cell + 6*t + e joins vertices
 * PAIR[e][0] and PAIR[e][1] of tetrahedron t.  Returns 0 or -1. */
static int build_pyro(orc *h)
{
    int L = h->L;
    int64_t ncell = (int64_t)L * L * L;
    h->N = 16 * ncell;
    h->NB = 48 * ncell;
    h->ba = (int32_t *)malloc(sizeof(int32_t) * h->NB);
    h->bb = (int32_t *)malloc(sizeof(int32_t) * h->NB);
    if (!h->ba || !h->bb) return -1;
    for (int64_t z = 0; z < L; ++z)
        for (int64_t y = 0; y < L; ++y)
            for (int64_t x = 0; x < L; ++x) {
                int64_t cell = (z * L + y) * L + x;
                for (int t = 0; t < 8; ++t) {
                    int f = t & 3, sgn = (t < 4) ? 1 : -1;
                    int64_t v[4];
                    for (int mu = 0; mu < 4; ++mu) {
                        int64_t p[3] = {4 * x + FCC[f][0] + sgn * BAS[mu][0],
                                        4 * y + FCC[f][1] + sgn * BAS[mu][1],
                                        4 * z + FCC[f][2] + sgn * BAS[mu][2]};
                        v[mu] = pyro_site_at(L, p);
                        if (v[mu] < 0) return -1;
                    }
                    for (int e = 0; e < 6; ++e) {
                        int64_t b = 48 * cell + 6 * t + e;
                        h->ba[b] = (int32_t)v[PAIR[e][0]];
                        h->bb[b] = (int32_t)v[PAIR[e][1]];
                    }
                }
            }
    return 0;
}

/* Simple cubic: site (z*L + y)*L + x, bond 3*i + d to the +d neighbour. */
static int build_sc(orc *h)
{
    int64_t L = h->L;
    h->N = L * L * L;
    h->NB = 3 * h->N;
    h->ba = (int32_t *)malloc(sizeof(int32_t) * h->NB);
    h->bb = (int32_t *)malloc(sizeof(int32_t) * h->NB);
    if (!h->ba || !h->bb) return -1;
    for (int64_t z = 0; z < L; ++z)
        for (int64_t y = 0; y < L; ++y)
            for (int64_t x = 0; x < L; ++x) {
                int64_t i = (z * L + y) * L + x;
                int64_t nb[3] = {(z * L + y) * L + (x + 1) % L,
                                 (z * L + (y + 1) % L) * L + x,
                                 (((z + 1) % L) * L + y) * L + x};
                for (int d = 0; d < 3; ++d) {
                    h->ba[3 * i + d] = (int32_t)i;
                    h->bb[3 * i + d] = (int32_t)nb[d];
                }
            }
    return 0;
}

static int build_adjacency(orc *h)
{
    h->adj_off = (int64_t *)calloc((size_t)h->N + 1, sizeof(int64_t));
    h->adj_bond = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)h->NB + 1);
    if (!h->adj_off || !h->adj_bond) return -1;
    for (int64_t b = 0; b < h->NB; ++b) {
        h->adj_off[h->ba[b] + 1]++;
        h->adj_off[h->bb[b] + 1]++;
    }
    for (int64_t i = 0; i < h->N; ++i) h->adj_off[i + 1] += h->adj_off[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)h->N + 1));
    if (!fill) return -1;
    memcpy(fill, h->adj_off, sizeof(int64_t) * (size_t)h->N);
    for (int64_t b = 0; b < h->NB; ++b) {
        h->adj_bond[fill[h->ba[b]]++] = b;
        h->adj_bond[fill[h->bb[b]]++] = b;
    }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Handle                                                                    */
/* ------------------------------------------------------------------------ */

void orc_destroy(orc *h)
{
    if (!h) return;
    free(h->ba); free(h->bb); free(h->adj_off); free(h->adj_bond);
    free(h->s8); free(h->sv); free(h->sigma); free(h->active);
    free(h->label); free(h->queue); free(h->flip);
    free(h);
}

static void set_params(orc *h, double T, double J)
{
    double twobj = 2.0 * J / T;
    if (h->plant == PLANT_HALF_BETA) twobj = J / T;
    h->T = T;
    h->J = J;
    h->thr = (uint64_t)floor(-expm1(-twobj) * 4294967296.0);
    h->x0 = (float)twobj;
}

void orc_set_temperature(orc *h, double T) { set_params(h, T, h->J); }

void orc_set_plant(orc *h, int plant)
{
    h->plant = plant;
    set_params(h, h->T, h->J);
}

static void initial_state(orc *h)
{
    if (h->model == ORC_ISING) {
        for (int64_t i = 0; i < h->N; ++i) {
            if (h->start == 0) {
                h->s8[i] = 1;
            } else {
                uint32_t w[4];
                draw(h->seed, (uint64_t)i >> 7, 0, ST_INIT, 0, w);
                int bit = (int)((w[(i >> 5) & 3] >> (i & 31)) & 1u);
                h->s8[i] = bit ? -1 : 1;
            }
        }
    } else {
        for (int64_t i = 0; i < h->N; ++i) {
            float v[3] = {1.0f, 0.0f, 0.0f};
            if (h->start != 0) unit_vector(h->seed, (uint64_t)i, 0, ST_INIT, h->n, v);
            for (int k = 0; k < h->n; ++k) h->sv[i * h->n + k] = v[k];
        }
    }
}

static int finish_create(orc *h, int model, double T, double J, uint64_t seed, int start)
{
    h->model = model;
    h->n = model;
    h->seed = seed;
    h->start = start;
    h->J = J;
    set_params(h, T, J);
    if (build_adjacency(h)) return -1;
    if (model == ORC_ISING) h->s8 = (int8_t *)malloc((size_t)h->N);
    else {
        h->sv = (float *)malloc(sizeof(float) * (size_t)h->N * h->n);
        h->sigma = (float *)malloc(sizeof(float) * (size_t)h->N);
    }
    h->active = (uint8_t *)calloc((size_t)h->NB + 1, 1);
    h->label = (int32_t *)malloc(sizeof(int32_t) * (size_t)h->N);
    h->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)h->N);
    h->flip = (uint8_t *)malloc((size_t)h->N);
    if ((model == ORC_ISING && !h->s8) || (model != ORC_ISING && (!h->sv || !h->sigma)) ||
        !h->active || !h->label || !h->queue || !h->flip)
        return -1;
    for (int64_t i = 0; i < h->N; ++i) h->label[i] = (int32_t)i;
    initial_state(h);
    h->t = 0;
    return 0;
}

static int check_args(int model, double T, double J, int start)
{
    if (model < 1 || model > 3) return -1;
    if (!(T > 0.0)) return -1; /* rejects NaN and T <= 0; T = +inf allowed */
    if (!(J > 0.0) || isinf(J)) return -1;
    if (start != 0 && start != 1) return -1;
    return 0;
}

int orc_create_pyro(orc **out, int L, int model, double T, double J, uint64_t seed, int start)
{
    *out = NULL;
    if (L < 1 || L > 200 || check_args(model, T, J, start)) return -1;
    orc *h = (orc *)calloc(1, sizeof(orc));
    if (!h) return -1;
    h->kind = ORC_KIND_PYRO;
    h->L = L;
    if (build_pyro(h) || finish_create(h, model, T, J, seed, start)) { orc_destroy(h); return -1; }
    *out = h;
    return 0;
}

int orc_create_sc(orc **out, int L, int model, double T, double J, uint64_t seed, int start)
{
    *out = NULL;
    if (L < 2 || L > 400 || check_args(model, T, J, start)) return -1;
    orc *h = (orc *)calloc(1, sizeof(orc));
    if (!h) return -1;
    h->kind = ORC_KIND_SC;
    h->L = L;
    if (build_sc(h) || finish_create(h, model, T, J, seed, start)) { orc_destroy(h); return -1; }
    *out = h;
    return 0;
}

/* Any graph given as an edge list (bond b joins a[b] and b[b]). */
int orc_create_edges(orc **out, int64_t N, int64_t NB, const int32_t *a, const int32_t *b,
                     int model, double T, double J, uint64_t seed, int start)
{
    *out = NULL;
    if (N < 1 || NB < 0 || check_args(model, T, J, start)) return -1;
    for (int64_t k = 0; k < NB; ++k)
        if (a[k] < 0 || a[k] >= N || b[k] < 0 || b[k] >= N || a[k] == b[k]) return -1;
    orc *h = (orc *)calloc(1, sizeof(orc));
    if (!h) return -1;
    h->kind = ORC_KIND_EDGES;
    h->N = N;
    h->NB = NB;
    h->ba = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NB + 1));
    h->bb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NB + 1));
    if (!h->ba || !h->bb) { orc_destroy(h); return -1; }
    memcpy(h->ba, a, sizeof(int32_t) * (size_t)NB);
    memcpy(h->bb, b, sizeof(int32_t) * (size_t)NB);
    if (finish_create(h, model, T, J, seed, start)) { orc_destroy(h); return -1; }
    *out = h;
    return 0;
}

int64_t orc_num_sites(const orc *h) { return h->N; }
int64_t orc_num_bonds(const orc *h) { return h->NB; }
int64_t orc_sweep_index(const orc *h) { return h->t; }
uint64_t orc_threshold(const orc *h) { return h->thr; }
float orc_x0(const orc *h) { return h->x0; }

void orc_bonds(const orc *h, int32_t *a, int32_t *b)
{
    memcpy(a, h->ba, sizeof(int32_t) * (size_t)h->NB);
    memcpy(b, h->bb, sizeof(int32_t) * (size_t)h->NB);
}

/* Spins in the exchange layout: Ising int8 [N]; O(n) float component-major
 * [n][N]. */
void orc_get_spins(const orc *h, void *dst)
{
    if (h->model == ORC_ISING) {
        memcpy(dst, h->s8, (size_t)h->N);
    } else {
        float *d = (float *)dst;
        for (int k = 0; k < h->n; ++k)
            for (int64_t i = 0; i < h->N; ++i) d[k * h->N + i] = h->sv[i * h->n + k];
    }
}

void orc_set_spins(orc *h, const void *src, int64_t sweep_index)
{
    if (h->model == ORC_ISING) {
        memcpy(h->s8, src, (size_t)h->N);
    } else {
        const float *s = (const float *)src;
        for (int k = 0; k < h->n; ++k)
            for (int64_t i = 0; i < h->N; ++i) h->sv[i * h->n + k] = s[k * h->N + i];
    }
    h->t = sweep_index;
}

void orc_get_labels(const orc *h, int32_t *dst) { memcpy(dst, h->label, sizeof(int32_t) * (size_t)h->N); }
void orc_get_active(const orc *h, uint8_t *dst) { memcpy(dst, h->active, (size_t)h->NB); }

/* ------------------------------------------------------------------------ */
/* Cluster labeling: connected components of the active-bond graph by       */
/* breadth-first search from each unlabeled site in increasing index order, */
/* so that every site receives the smallest site index of its cluster.      */
/* ------------------------------------------------------------------------ */
static void label_clusters(orc *h)
{
    for (int64_t i = 0; i < h->N; ++i) h->label[i] = -1;
    for (int64_t i = 0; i < h->N; ++i) {
        if (h->label[i] >= 0) continue;
        h->label[i] = (int32_t)i;
        int64_t head = 0, tail = 0;
        h->queue[tail++] = (int32_t)i;
        while (head < tail) {
            int32_t v = h->queue[head++];
            for (int64_t k = h->adj_off[v]; k < h->adj_off[v + 1]; ++k) {
                int64_t b = h->adj_bond[k];
                if (!h->active[b]) continue;
                int32_t w = (h->ba[b] == v) ? h->bb[b] : h->ba[b];
                if (h->label[w] < 0) {
                    h->label[w] = (int32_t)i;
                    h->queue[tail++] = w;
                }
            }
        }
    }
}

/* Stand-alone component labeling for tests. */
void orc_label_components(int64_t N, int64_t NB, const int32_t *a, const int32_t *b,
                          const uint8_t *active, int32_t *label)
{
    orc h;
    memset(&h, 0, sizeof(h));
    h.N = N;
    h.NB = NB;
    h.ba = (int32_t *)a;
    h.bb = (int32_t *)b;
    h.active = (uint8_t *)active;
    h.label = label;
    h.queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    if (build_adjacency(&h) == 0) label_clusters(&h);
    free(h.queue);
    free(h.adj_off);
    free(h.adj_bond);
}

static void choose_flips(orc *h)
{
    for (int64_t i = 0; i < h->N; ++i) {
        if (h->label[i] != i) continue;
        h->flip[i] = (h->plant == PLANT_FLIP_ALL) ? 1 : (uint8_t)flip_bit(h->seed, (uint64_t)i, h->t);
    }
}

static void record(const orc *h, orc_record *r)
{
    memset(r, 0, sizeof(*r));
    r->sweep = h->t;
    double m;
    if (h->model == ORC_ISING) {
        int64_t M = 0, B = 0;
        for (int64_t i = 0; i < h->N; ++i) M += h->s8[i];
        for (int64_t b = 0; b < h->NB; ++b) B += (int64_t)h->s8[h->ba[b]] * h->s8[h->bb[b]];
        r->bond_sum = B;
        r->M_int = M;
        r->E = -h->J * (double)B;
        r->M[0] = (double)M;
        m = (double)M / (double)h->N;
    } else {
        double M[3] = {0.0, 0.0, 0.0}, S = 0.0;
        for (int64_t i = 0; i < h->N; ++i)
            for (int k = 0; k < h->n; ++k) M[k] += (double)h->sv[i * h->n + k];
        for (int64_t b = 0; b < h->NB; ++b) {
            const float *sa = h->sv + (int64_t)h->ba[b] * h->n;
            const float *sb = h->sv + (int64_t)h->bb[b] * h->n;
            double d = 0.0;
            for (int k = 0; k < h->n; ++k) d += (double)sa[k] * (double)sb[k];
            S += d;
        }
        r->E = -h->J * S;
        for (int k = 0; k < 3; ++k) r->M[k] = M[k];
        m = sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]) / (double)h->N;
    }
    r->m2 = m * m;
    r->m4 = r->m2 * r->m2;
}

/* One Ising sweep. */
static void sweep_ising(orc *h)
{
    for (int64_t b = 0; b < h->NB; ++b) {
        int8_t sa = h->s8[h->ba[b]], sb = h->s8[h->bb[b]];
        /* A vacant site (spin 0, site dilution) carries no bond: a bond is a
         * candidate only when both ends hold equal nonzero spins. */
        int parallel = (h->plant == PLANT_ANTI) ? (sa != sb)
                                                 : (sa == sb && (sa != 0 || h->plant == PLANT_VACANT_JOIN));
        uint8_t act = 0;
        if (parallel) act = (uint64_t)ising_bond_uniform(h->seed, (uint64_t)b, h->t) < h->thr;
        if (h->plant == PLANT_DROP_BONDS && (b & 1)) act = 0;
        h->active[b] = act;
    }
    label_clusters(h);
    choose_flips(h);
    for (int64_t i = 0; i < h->N; ++i)
        if (h->flip[h->label[i]]) h->s8[i] = (int8_t)-h->s8[i];
}

/* One O(n) sweep with Wolff's embedding: project every spin on one random
 * axis r, run the Ising-like cluster construction on the projections, and
 * reflect the flipped clusters through the plane normal to r. */
static void sweep_on(orc *h)
{
    int n = h->n;
    float r[3];
    orc_axis(h->seed, h->t, n, r);
    for (int64_t i = 0; i < h->N; ++i) {
        const float *s = h->sv + i * n;
        float sig = s[0] * r[0];
        sig = fmaf(s[1], r[1], sig);
        if (n == 3) sig = fmaf(s[2], r[2], sig);
        h->sigma[i] = sig;
    }
    for (int64_t b = 0; b < h->NB; ++b) {
        float x = (h->x0 * h->sigma[h->ba[b]]) * h->sigma[h->bb[b]];
        uint32_t r32 = on_bond_uniform(h->seed, (uint64_t)b, h->t);
        double u = ((double)r32 + 0.5) * 0x1p-32;
        uint8_t act = (double)x > -log1p(-u);
        if (h->plant == PLANT_DROP_BONDS && (b & 1)) act = 0;
        h->active[b] = act;
    }
    label_clusters(h);
    choose_flips(h);
    for (int64_t i = 0; i < h->N; ++i) {
        if (!h->flip[h->label[i]]) continue;
        float *s = h->sv + i * n;
        float c = (h->plant == PLANT_REFLECT_SIGN) ? 2.0f * h->sigma[i] : -2.0f * h->sigma[i];
        for (int k = 0; k < n; ++k) s[k] = fmaf(c, r[k], s[k]);
    }
}

/* Run n_sweeps sweeps; write one record per sweep (state after the sweep)
 * into rec[0..n_sweeps-1] when rec is not NULL. */
int orc_sweep(orc *h, int64_t n_sweeps, orc_record *rec)
{
    if (n_sweeps < 0) return -1;
    for (int64_t k = 0; k < n_sweeps; ++k) {
        if (h->model == ORC_ISING) sweep_ising(h);
        else sweep_on(h);
        if (rec) record(h, &rec[k]);
        h->t++;
    }
    return 0;
}

/* Record of the current state without sweeping (sweep index = t - 1). */
void orc_measure(const orc *h, orc_record *r)
{
    record(h, r);
    r->sweep = h->t - 1;
}
