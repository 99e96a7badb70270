/* Sanitizer driver of the CPU oracle (test infrastructure): exercises every
 * entry point of oracle/pyro_oracle.c on small lattices of all three models
 * (pyrochlore L = 1..3, simple cubic, an edge list, site dilution) so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build reports any invalid
 * access or undefined operation.  Prints "oracle sanitize ok" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc orc;
typedef struct {
    int64_t sweep, bond_sum, M_int, pad;
    double E, M[3], m2, m4;
} orc_record;

int orc_create_pyro(orc **out, int L, int model, double T, double J, uint64_t seed, int start);
int orc_create_sc(orc **out, int L, int model, double T, double J, uint64_t seed, int start);
int orc_create_edges(orc **out, int64_t N, int64_t NB, const int32_t *a, const int32_t *b, int model, double T,
                     double J, uint64_t seed, int start);
void orc_destroy(orc *h);
int orc_sweep(orc *h, int64_t n_sweeps, orc_record *rec);
void orc_measure(const orc *h, orc_record *r);
int64_t orc_num_sites(const orc *h);
int64_t orc_num_bonds(const orc *h);
void orc_bonds(const orc *h, int32_t *a, int32_t *b);
void orc_get_spins(const orc *h, void *dst);
void orc_set_spins(orc *h, const void *src, int64_t sweep_index);
void orc_get_labels(const orc *h, int32_t *dst);
void orc_get_active(const orc *h, uint8_t *dst);
void orc_set_temperature(orc *h, double T);
void orc_label_components(int64_t N, int64_t NB, const int32_t *a, const int32_t *b, const uint8_t *active,
                          int32_t *label);
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_axis(uint64_t seed, int64_t t, int n, float r[3]);
uint64_t orc_ising_threshold(double T, double J);
void orc_pyro_position(int L, int64_t i, int32_t pos[3]);

static int exercise(orc *h, int model, int dilute)
{
    const int64_t N = orc_num_sites(h), NB = orc_num_bonds(h);
    const int n = model;
    orc_record rec[40];
    if (orc_sweep(h, 20, rec) != 0) return 1;
    int32_t *a = malloc(sizeof(int32_t) * (size_t)NB), *b = malloc(sizeof(int32_t) * (size_t)NB);
    int32_t *lab = malloc(sizeof(int32_t) * (size_t)N), *lab2 = malloc(sizeof(int32_t) * (size_t)N);
    uint8_t *act = malloc((size_t)NB);
    const size_t sb = model == 1 ? (size_t)N : sizeof(float) * (size_t)(n * N);
    void *s = malloc(sb);
    orc_bonds(h, a, b);
    orc_get_labels(h, lab);
    orc_get_active(h, act);
    orc_label_components(N, NB, a, b, act, lab2);
    int bad = memcmp(lab, lab2, sizeof(int32_t) * (size_t)N) != 0;
    orc_get_spins(h, s);
    if (dilute) { /* every third site vacant */
        for (int64_t i = 0; i < N; i += 3) {
            if (model == 1) ((int8_t *)s)[i] = 0;
            else for (int k = 0; k < n; ++k) ((float *)s)[k * N + i] = 0.0f;
        }
    }
    orc_set_spins(h, s, 1000);
    orc_set_temperature(h, INFINITY);
    orc_sweep(h, 5, rec);
    orc_set_temperature(h, 1e-3);
    orc_sweep(h, 5, rec);
    orc_measure(h, &rec[0]);
    free(a); free(b); free(lab); free(lab2); free(act); free(s);
    return bad;
}

int main(void)
{
    int fails = 0;
    for (int L = 1; L <= 3; ++L)
        for (int model = 1; model <= 3; ++model)
            for (int dil = 0; dil < 2; ++dil) {
                orc *h = NULL;
                if (orc_create_pyro(&h, L, model, model == 1 ? 4.2139 : 1.5, 1.0, 7 + L, L & 1) != 0) return 2;
                fails += exercise(h, model, dil);
                orc_destroy(h);
            }
    for (int model = 1; model <= 3; ++model) {
        orc *h = NULL;
        if (orc_create_sc(&h, 3, model, 4.5, 1.0, 3, 1) != 0) return 3;
        fails += exercise(h, model, 0);
        orc_destroy(h);
    }
    {
        const int32_t ea[5] = {0, 1, 2, 3, 0}, eb[5] = {1, 2, 3, 4, 4};
        orc *h = NULL;
        if (orc_create_edges(&h, 6, 5, ea, eb, 2, 1.0, 1.0, 5, 1) != 0) return 4;
        fails += exercise(h, 2, 1);
        orc_destroy(h);
    }
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox(ctr, key, out);
    float r[3];
    orc_axis(9, 17, 3, r);
    (void)orc_ising_threshold(4.2139, 1.0);
    (void)orc_ising_threshold(INFINITY, 1.0);
    int32_t pos[3];
    orc_pyro_position(2, 127, pos);
    if (fails) {
        fprintf(stderr, "labels differ from connected components in %d runs\n", fails);
        return 1;
    }
    printf("oracle sanitize ok\n");
    return 0;
}
