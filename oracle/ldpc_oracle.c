/*
 * CPU oracle: quantized layered belief-propagation decoding of LDPC syndromes,
 * after Mao, Li, Han, Guo, "High Throughput and Low Cost LDPC Reconciliation
 * for Quantum Key Distribution" (arXiv:1903.10107).
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow, step-by-step statement of
 * what the decoder computes. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may call it; the product library never links it.
 * It shares no code, header, table or helper with the HIP library: it builds
 * its own parity-check structure from the base matrix.
 *
 * Integer conventions (the paper leaves these open; each is one reading):
 *   - soft values E are clamped symmetrically to [-E_max, E_max]; -128 never
 *     occurs (the freeze test |E| == E_max of Alg. 2 is then symmetric);
 *   - the VN->CN message L_ji = E_j - L_ij (Eq. 8) is saturated to the
 *     accumulator range: +-127 with 8-bit soft values, +-32767 with 16-bit;
 *   - the sign of a message is its two's-complement sign bit, so 0 is positive,
 *     and the hard decision of VN j is [E_j < 0];
 *   - syndrome decoding: the check-node sign (Eq. 1) is multiplied by
 *     (-1)^{s_i}, and a frame has converged when H x^ = s;
 *   - initial state E_j = llr_j, every L_ij = 0; the syndrome is tested before
 *     the first iteration (iteration count 0) and after every full iteration;
 *   - layers in ascending base-row order; within a row the edges are taken in
 *     ascending base-column order; block (b, c) with shift s joins row b*Z + r
 *     to column c*Z + (r + s) mod Z;
 *   - the degree-d box-plus of Eq. 4, evaluated with the integer tau of Alg. 1
 *     which is not associative, uses the forward-backward order (rule 0); the
 *     literal right fold of Eq. 7 is rule 1; min-sum is rule 2.
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC (see build.py beside this file).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_RULE_RCBP_FB 0
#define ORACLE_RULE_RCBP_EQ7 1
#define ORACLE_RULE_MINSUM 2

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static int iabs(int a) { return a < 0 ? -a : a; }
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Check node: Alg. 1 (Sec. 3.2), the integer table tau(p, q) that stands for */
/* beta((p + 1/2) Delta, (q + 1/2) Delta) of Eq. 6, computed by formula.       */
/*                                                                            */
/* Read as a correction: the box-plus of two magnitudes (each first clipped  */
/* to msg_max) is the smaller one, lowered by one step for every closeness    */
/* threshold that the gap between the two stays below, and never below 0.    */
/* A smaller operand above 2 has the thresholds 2 and 6 (up to two steps); a  */
/* smaller operand of 2 or less has the single threshold 4.                   */
/* ------------------------------------------------------------------------ */
static const int tau_gap_thresholds_large[] = {2, 6};
static const int tau_gap_thresholds_small[] = {4};

int oracle_tau(int p, int q, int msg_max)
{
    const int lo = imin(imin(p, q), msg_max);
    const int hi = imin(imax(p, q), msg_max);
    const int gap = hi - lo;
    const int *th = lo > 2 ? tau_gap_thresholds_large : tau_gap_thresholds_small;
    const int n_th = lo > 2 ? 2 : 1;
    int steps = 0;
    for (int i = 0; i < n_th; i++)
        if (gap < th[i])
            steps++;
    return imax(lo - steps, 0);
}

/* Degree-d box-plus of every "all operands but k" subset (Eq. 4), with tau as
 * the two-operand box-plus, in forward-backward order:
 *   F_0 = p_0, F_k = tau(F_{k-1}, p_k);  B_{d-1} = p_{d-1}, B_k = tau(p_k, B_{k+1})
 *   mag_0 = B_1, mag_{d-1} = F_{d-2}, mag_k = tau(F_{k-1}, B_{k+1}).
 * A single remaining operand (d = 2) is passed through clipped to msg_max. */
void oracle_cn_rcbp_fb(const int *p, int d, int msg_max, int *mag)
{
    int F[512], B[512];
    if (d < 2 || d > 512)
        return;
    F[0] = p[0];
    for (int k = 1; k < d; k++)
        F[k] = oracle_tau(F[k - 1], p[k], msg_max);
    B[d - 1] = p[d - 1];
    for (int k = d - 2; k >= 0; k--)
        B[k] = oracle_tau(p[k], B[k + 1], msg_max);
    mag[0] = imin(B[1], msg_max);
    mag[d - 1] = imin(F[d - 2], msg_max);
    for (int k = 1; k < d - 1; k++)
        mag[k] = oracle_tau(F[k - 1], B[k + 1], msg_max);
}

/* The same subsets folded literally as Eq. 7 prints it: the operands other
 * than k, in ascending edge order o_1 < ... < o_{d-1}, as
 *   beta(p_{o_1}, beta(p_{o_2}, ..., beta(p_{o_{d-2}}, p_{o_{d-1}}))). */
void oracle_cn_rcbp_eq7(const int *p, int d, int msg_max, int *mag)
{
    int ops[512];
    if (d < 2 || d > 512)
        return;
    for (int k = 0; k < d; k++) {
        int m = 0;
        for (int i = 0; i < d; i++)
            if (i != k)
                ops[m++] = p[i];
        int acc = imin(ops[m - 1], msg_max);
        for (int i = m - 2; i >= 0; i--)
            acc = oracle_tau(ops[i], acc, msg_max);
        mag[k] = acc;
    }
}

/* Min-sum: the smallest magnitude among the other operands, clipped. */
void oracle_cn_minsum(const int *p, int d, int msg_max, int *mag)
{
    for (int k = 0; k < d; k++) {
        int m = msg_max;
        for (int i = 0; i < d; i++)
            if (i != k)
                m = imin(m, p[i]);
        mag[k] = m;
    }
}

static void cn_magnitudes(int rule, const int *p, int d, int msg_max, int *mag)
{
    if (rule == ORACLE_RULE_RCBP_EQ7)
        oracle_cn_rcbp_eq7(p, d, msg_max, mag);
    else if (rule == ORACLE_RULE_MINSUM)
        oracle_cn_minsum(p, d, msg_max, mag);
    else
        oracle_cn_rcbp_fb(p, d, msg_max, mag);
}

/* ------------------------------------------------------------------------ */
/* Variable node: Eq. 9 under the saturation rule of Alg. 2 (Sec. 3.3).       */
/* e: the stored soft value E_j; v: the VN->CN message L_ji = E_j - L_ij^{t-1}  */
/* (Eq. 8, already saturated); lnew: the new CN->VN message L_ij^t.            */
/* With freeze set, a soft value already at +-e_max is left as it is.          */
/* ------------------------------------------------------------------------ */
int oracle_vn_update(int e, int v, int lnew, int e_max, int freeze)
{
    if (freeze && iabs(e) == e_max)
        return e;
    return clampi(v + lnew, -e_max, e_max);
}

/* ------------------------------------------------------------------------ */
/* Parity-check structure, built here from the base matrix on its own.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int mb, nb, z;
    int n, m;
    int n_blocks;
    int *deg;       /* [mb] nonzero blocks in base row b */
    int *blk_off;   /* [mb] index of base row b's first block */
    int *blk_col;   /* [n_blocks] base column, ascending within a row */
    int *blk_shift; /* [n_blocks] circulant shift */
} oracle_graph;

static int graph_build(oracle_graph *g, const int32_t *base, int mb, int nb, int z)
{
    memset(g, 0, sizeof(*g));
    g->mb = mb; g->nb = nb; g->z = z;
    g->n = nb * z; g->m = mb * z;
    int nblk = 0;
    for (int i = 0; i < mb * nb; i++)
        if (base[i] >= 0)
            nblk++;
    g->n_blocks = nblk;
    g->deg = calloc((size_t)mb, sizeof(int));
    g->blk_off = calloc((size_t)mb, sizeof(int));
    g->blk_col = calloc((size_t)(nblk ? nblk : 1), sizeof(int));
    g->blk_shift = calloc((size_t)(nblk ? nblk : 1), sizeof(int));
    if (!g->deg || !g->blk_off || !g->blk_col || !g->blk_shift)
        return -1;
    int e = 0;
    for (int b = 0; b < mb; b++) {
        g->blk_off[b] = e;
        for (int c = 0; c < nb; c++) {
            int s = base[b * nb + c];
            if (s >= 0) {
                g->blk_col[e] = c;
                g->blk_shift[e] = s;
                e++;
            }
        }
        g->deg[b] = e - g->blk_off[b];
    }
    return 0;
}

static void graph_free(oracle_graph *g)
{
    free(g->deg); free(g->blk_off); free(g->blk_col); free(g->blk_shift);
}

/* VN index of row r of block blk */
static int edge_vn(const oracle_graph *g, int blk, int r)
{
    return g->blk_col[blk] * g->z + (r + g->blk_shift[blk]) % g->z;
}

/* H x^ == s, with x^_j = [E_j < 0] */
static int syndrome_ok(const oracle_graph *g, const int *E, const uint8_t *syn_bits)
{
    for (int b = 0; b < g->mb; b++) {
        for (int r = 0; r < g->z; r++) {
            int par = syn_bits[b * g->z + r];
            for (int k = 0; k < g->deg[b]; k++)
                par ^= (E[edge_vn(g, g->blk_off[b] + k, r)] < 0);
            if (par)
                return 0;
        }
    }
    return 1;
}

typedef struct {
    int32_t msg_max;      /* MSGmax of Alg. 1 */
    int32_t e_max;        /* E_max of Alg. 2 */
    int32_t acc_bits;     /* 8 or 16: width of the soft values */
    int32_t cn_rule;      /* ORACLE_RULE_* */
    const int8_t *offset; /* [offset_iters][n_blocks] magnitude offsets, or NULL */
    int32_t offset_iters;
    int32_t freeze;       /* 1: Alg. 2 saturation rule; 0: plain Eq. 9 */
} oracle_params;

/* One frame. Returns the iteration count; *conv is 1 iff H x^ = s at the end.
 * L_out: [n_blocks][z] int8 or NULL; E_out: [n] int16 or NULL. */
static int decode_frame(const oracle_graph *g, const oracle_params *prm,
                        const uint8_t *syn_packed, const int8_t *llr, int max_iter,
                        uint8_t *bits_out, uint8_t *conv_out, int8_t *L_out, int16_t *E_out)
{
    const int n = g->n, m = g->m, z = g->z;
    const int acc_lim = prm->acc_bits == 16 ? 32767 : 127;
    const int e_max = prm->e_max;
    const int init_lim = imin(127, e_max);
    int *E = malloc(sizeof(int) * (size_t)n);
    int *L = calloc((size_t)g->n_blocks * (size_t)z, sizeof(int));
    uint8_t *syn = malloc((size_t)m);
    int v[512], p[512], mag[512];

    for (int i = 0; i < m; i++)
        syn[i] = (syn_packed[i >> 3] >> (i & 7)) & 1;
    for (int j = 0; j < n; j++)
        E[j] = clampi(llr[j], -init_lim, init_lim);

    int conv = syndrome_ok(g, E, syn);
    int iters = 0;
    for (int t = 1; t <= max_iter && !conv; t++) {
        for (int b = 0; b < g->mb; b++) {
            const int d = g->deg[b];
            const int off0 = g->blk_off[b];
            for (int r = 0; r < z; r++) {
                /* Eq. 8: VN->CN messages, and the sign product of Eq. 1 times the syndrome bit */
                int parity = syn[b * z + r];
                for (int k = 0; k < d; k++) {
                    int j = edge_vn(g, off0 + k, r);
                    v[k] = clampi(E[j] - L[(off0 + k) * z + r], -acc_lim, acc_lim);
                    parity ^= (v[k] < 0);
                    p[k] = imin(iabs(v[k]), prm->msg_max);
                }
                /* magnitudes of Eq. 4 over all operands but k */
                cn_magnitudes(prm->cn_rule, p, d, prm->msg_max, mag);
                for (int k = 0; k < d; k++) {
                    int blk = off0 + k;
                    int mg = mag[k];
                    if (prm->offset && prm->offset_iters > 0) {
                        int ti = imin(t - 1, prm->offset_iters - 1);
                        mg = clampi(mg - prm->offset[ti * g->n_blocks + blk], 0, prm->msg_max);
                    }
                    /* Eq. 1: sign of the product over the other operands and the syndrome */
                    int lnew = (parity ^ (v[k] < 0)) ? -mg : mg;
                    int j = edge_vn(g, blk, r);
                    /* Eq. 9 with the saturation rule of Alg. 2 */
                    E[j] = oracle_vn_update(E[j], v[k], lnew, e_max, prm->freeze);
                    L[blk * z + r] = lnew;
                }
            }
        }
        iters = t;
        conv = syndrome_ok(g, E, syn);
    }
    if (!conv)
        iters = max_iter;

    memset(bits_out, 0, (size_t)(n + 7) / 8);
    for (int j = 0; j < n; j++)
        if (E[j] < 0)
            bits_out[j >> 3] |= (uint8_t)(1u << (j & 7));
    *conv_out = (uint8_t)conv;
    if (L_out)
        for (long e = 0; e < (long)g->n_blocks * z; e++)
            L_out[e] = (int8_t)L[e];
    if (E_out)
        for (int j = 0; j < n; j++)
            E_out[j] = (int16_t)E[j];
    free(E); free(L); free(syn);
    return iters;
}

/* Batch of frames. Returns 0, or -1 on invalid arguments.
 * syn: [F][ceil(m/8)] packed LSB-first; llr: [F][n]; out_bits: [F][ceil(n/8)];
 * out_conv: [F]; out_iters: [F] or NULL; out_L: [F][n_blocks][z] or NULL;
 * out_E: [F][n] (int16) or NULL. n_threads <= 0 uses the OpenMP default. */
int oracle_decode(const int32_t *base, int mb, int nb, int z, const oracle_params *prm,
                  const uint8_t *syn, const int8_t *llr, int n_frames, int max_iter,
                  uint8_t *out_bits, uint8_t *out_conv, int32_t *out_iters,
                  int8_t *out_L, int16_t *out_E, int n_threads)
{
    oracle_graph g;
    if (!base || !prm || mb < 1 || nb < 1 || z < 1 || n_frames < 0 || max_iter < 0)
        return -1;
    if (prm->acc_bits != 8 && prm->acc_bits != 16)
        return -1;
    if (prm->e_max < 1 || prm->e_max > (prm->acc_bits == 16 ? 32767 : 127))
        return -1;
    if (prm->msg_max < 1 || prm->msg_max > 127)
        return -1;
    if (graph_build(&g, base, mb, nb, z) != 0)
        return -1;
    for (int b = 0; b < mb; b++)
        if (g.deg[b] < 2 || g.deg[b] > 512) {
            graph_free(&g);
            return -1;
        }
    const size_t sb = (size_t)(g.m + 7) / 8, nbits = (size_t)(g.n + 7) / 8;
    const size_t ne = (size_t)g.n_blocks * (size_t)z;
#ifdef _OPENMP
    /* a thread count for this call only (a num_threads clause, not the
     * process-wide default, so a one-thread call leaves later calls alone) */
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int f = 0; f < n_frames; f++) {
        int it = decode_frame(&g, prm, syn + (size_t)f * sb, llr + (size_t)f * (size_t)g.n, max_iter,
                              out_bits + (size_t)f * nbits, out_conv + f,
                              out_L ? out_L + (size_t)f * ne : NULL,
                              out_E ? out_E + (size_t)f * (size_t)g.n : NULL);
        if (out_iters)
            out_iters[f] = it;
    }
    graph_free(&g);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* FP64 layered BP (Sec. 2): the floating-point decoder the quantized one     */
/* approximates. Used for frame error rate and efficiency statistics only.    */
/* ------------------------------------------------------------------------ */

/* Eq. 6 for magnitudes a, b >= 0, in the overflow-free form
 * min(a, b) + ln(1 + e^{-(a+b)}) - ln(1 + e^{-|a-b|}), which equals
 * 2 atanh(tanh(a/2) tanh(b/2)). */
double oracle_beta(double a, double b)
{
    return fmin(a, b) + log1p(exp(-(a + b))) - log1p(exp(-fabs(a - b)));
}

/* Eq. 2: 2 atanh of the product of tanh(|L|/2) over the operands but k */
double oracle_mag_tanh(const double *a, int d, int k)
{
    double prod = 1.0;
    for (int i = 0; i < d; i++)
        if (i != k)
            prod *= tanh(fabs(a[i]) / 2.0);
    return 2.0 * atanh(prod);
}

/* Eq. 3 with phi of Eq. 5 */
static double phi(double x) { return -log(tanh(x / 2.0)); }
double oracle_mag_phi(const double *a, int d, int k)
{
    double s = 0.0;
    for (int i = 0; i < d; i++)
        if (i != k)
            s += phi(fabs(a[i]));
    return phi(s);
}

/* Eq. 7: right fold of beta over the operands but k, ascending */
double oracle_mag_fold(const double *a, int d, int k)
{
    double acc = -1.0;
    for (int i = d - 1; i >= 0; i--) {
        if (i == k)
            continue;
        acc = acc < 0.0 ? fabs(a[i]) : oracle_beta(fabs(a[i]), acc);
    }
    return acc;
}

static int syndrome_ok_f(const oracle_graph *g, const double *E, const uint8_t *syn)
{
    for (int b = 0; b < g->mb; b++)
        for (int r = 0; r < g->z; r++) {
            int par = syn[b * g->z + r];
            for (int k = 0; k < g->deg[b]; k++)
                par ^= (E[edge_vn(g, g->blk_off[b] + k, r)] < 0.0);
            if (par)
                return 0;
        }
    return 1;
}

/* FP64 layered BP over a batch: same schedule and stopping rule as the integer
 * decoder; check node by the exact box-plus (forward-backward over beta). */
int oracle_bp_fp64_decode(const int32_t *base, int mb, int nb, int z,
                          const uint8_t *syn, const double *llr, int n_frames, int max_iter,
                          uint8_t *out_bits, uint8_t *out_conv, int32_t *out_iters, int n_threads)
{
    oracle_graph g;
    if (!base || mb < 1 || nb < 1 || z < 1 || n_frames < 0 || max_iter < 0)
        return -1;
    if (graph_build(&g, base, mb, nb, z) != 0)
        return -1;
    for (int b = 0; b < mb; b++)
        if (g.deg[b] < 2 || g.deg[b] > 512) {
            graph_free(&g);
            return -1;
        }
    const size_t sb = (size_t)(g.m + 7) / 8, nbits = (size_t)(g.n + 7) / 8;
#ifdef _OPENMP
    /* a thread count for this call only (a num_threads clause, not the
     * process-wide default, so a one-thread call leaves later calls alone) */
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int f = 0; f < n_frames; f++) {
        const int n = g.n, m = g.m;
        double *E = malloc(sizeof(double) * (size_t)n);
        double *L = calloc((size_t)g.n_blocks * (size_t)z, sizeof(double));
        uint8_t *sv = malloc((size_t)m);
        double v[512], F[512], B[512];
        const uint8_t *sp = syn + (size_t)f * sb;
        for (int i = 0; i < m; i++)
            sv[i] = (sp[i >> 3] >> (i & 7)) & 1;
        for (int j = 0; j < n; j++)
            E[j] = llr[(size_t)f * (size_t)n + (size_t)j];
        int conv = syndrome_ok_f(&g, E, sv), iters = 0;
        for (int t = 1; t <= max_iter && !conv; t++) {
            for (int b = 0; b < g.mb; b++) {
                const int d = g.deg[b], o = g.blk_off[b];
                for (int r = 0; r < z; r++) {
                    int parity = sv[b * z + r];
                    for (int k = 0; k < d; k++) {
                        v[k] = E[edge_vn(&g, o + k, r)] - L[(o + k) * z + r];
                        parity ^= (v[k] < 0.0);
                    }
                    F[0] = fabs(v[0]);
                    for (int k = 1; k < d; k++)
                        F[k] = oracle_beta(F[k - 1], fabs(v[k]));
                    B[d - 1] = fabs(v[d - 1]);
                    for (int k = d - 2; k >= 0; k--)
                        B[k] = oracle_beta(fabs(v[k]), B[k + 1]);
                    for (int k = 0; k < d; k++) {
                        double mg = k == 0 ? B[1] : (k == d - 1 ? F[d - 2] : oracle_beta(F[k - 1], B[k + 1]));
                        double ln = (parity ^ (v[k] < 0.0)) ? -mg : mg;
                        E[edge_vn(&g, o + k, r)] = v[k] + ln;
                        L[(o + k) * z + r] = ln;
                    }
                }
            }
            iters = t;
            conv = syndrome_ok_f(&g, E, sv);
        }
        if (!conv)
            iters = max_iter;
        uint8_t *bo = out_bits + (size_t)f * nbits;
        memset(bo, 0, nbits);
        for (int j = 0; j < n; j++)
            if (E[j] < 0.0)
                bo[j >> 3] |= (uint8_t)(1u << (j & 7));
        out_conv[f] = (uint8_t)conv;
        if (out_iters)
            out_iters[f] = iters;
        free(E); free(L); free(sv);
    }
    graph_free(&g);
    return 0;
}
