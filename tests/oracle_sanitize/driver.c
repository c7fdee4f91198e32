/*
 * Sanitizer driver for the CPU oracle (test infrastructure): links
 * oracle/ldpc_oracle.c into one executable built with AddressSanitizer and
 * UndefinedBehaviorSanitizer and runs its entry points over 8- and 16-bit soft
 * values, the three check-node rules, offset tables, the freeze switch,
 * channel values of -128 and the FP64 decoder. Any sanitizer report fails
 * the run (-fno-sanitize-recover).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t msg_max, e_max, acc_bits, cn_rule;
    const int8_t *offset;
    int32_t offset_iters, freeze;
} params;

int oracle_decode(const int32_t *base, int mb, int nb, int z, const params *prm, const uint8_t *syn,
                  const int8_t *llr, int n_frames, int max_iter, uint8_t *out_bits, uint8_t *out_conv,
                  int32_t *out_iters, int8_t *out_L, int16_t *out_E, int n_threads);
int oracle_bp_fp64_decode(const int32_t *base, int mb, int nb, int z, const uint8_t *syn, const double *llr,
                          int n_frames, int max_iter, uint8_t *out_bits, uint8_t *out_conv, int32_t *out_iters,
                          int n_threads);
int oracle_tau(int p, int q, int msg_max);

static uint32_t rng = 12345u;
static uint32_t next(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 17;
    rng ^= rng << 5;
    return rng;
}

int main(void)
{
    enum { MB = 3, NB = 8, Z = 16, F = 6 };
    int32_t base[MB * NB];
    for (int i = 0; i < MB * NB; i++)
        base[i] = (next() % 5 == 0 && i % NB > 2) ? -1 : (int32_t)(next() % Z);
    const int n = NB * Z, m = MB * Z;
    int nblk = 0;
    for (int i = 0; i < MB * NB; i++)
        nblk += base[i] >= 0;
    uint8_t *syn = calloc((size_t)F * ((m + 7) / 8), 1);
    int8_t *llr = malloc((size_t)F * n);
    double *llr_f = malloc(sizeof(double) * (size_t)F * n);
    for (int i = 0; i < F * ((m + 7) / 8); i++)
        syn[i] = (uint8_t)next();
    for (int i = 0; i < F * n; i++) {
        uint32_t r = next() % 16;
        llr[i] = r == 0 ? -128 : r == 1 ? 127 : (int8_t)((int)(next() % 41) - 20);
        llr_f[i] = llr[i] * 0.3125;
    }
    int8_t *off = malloc((size_t)3 * nblk);
    for (int i = 0; i < 3 * nblk; i++)
        off[i] = (int8_t)((int)(next() % 9) - 2);
    uint8_t *bits = malloc((size_t)F * ((n + 7) / 8)), conv[F];
    int32_t iters[F];
    int8_t *L = malloc((size_t)F * nblk * Z);
    int16_t *E = malloc(sizeof(int16_t) * (size_t)F * n);
    int runs = 0;
    for (int acc = 8; acc <= 16; acc += 8)
        for (int rule = 0; rule < 3; rule++)
            for (int with_off = 0; with_off < 2; with_off++)
                for (int freeze = 0; freeze < 2; freeze++) {
                    params p = {63, acc == 16 ? 200 : 100, acc, rule, with_off ? off : NULL, with_off ? 3 : 0,
                                freeze};
                    if (oracle_decode(base, MB, NB, Z, &p, syn, llr, F, 12, bits, conv, iters, L, E, 2) != 0) {
                        fprintf(stderr, "oracle_decode refused a valid call\n");
                        return 1;
                    }
                    runs++;
                }
    if (oracle_bp_fp64_decode(base, MB, NB, Z, syn, llr_f, F, 12, bits, conv, iters, 2) != 0)
        return 1;
    params bad = {63, 127, 12, 0, NULL, 0, 1};
    if (oracle_decode(base, MB, NB, Z, &bad, syn, llr, F, 5, bits, conv, iters, NULL, NULL, 1) != -1)
        return 1;
    long acc = 0;
    for (int a = 0; a < 70; a++)
        for (int b = 0; b < 70; b++)
            acc += oracle_tau(a, b, 63);
    printf("sanitized oracle runs: %d decodes, tau sum %ld\n", runs, acc);
    free(syn); free(llr); free(llr_f); free(off); free(bits); free(L); free(E);
    return 0;
}
