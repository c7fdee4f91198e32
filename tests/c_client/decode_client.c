/*
 * A plain C program that uses the decoder only through its C ABI
 * (include/qkdldpc.h) and the HIP runtime for device memory: no Python, no
 * torch. It reads a batch from a file, decodes it with ldpc_decode_batch_ex on
 * a stream of its own, and writes the results to a file; the GPU test suite
 * compares them with the CPU oracle.
 *
 * Input file (little-endian): int32 mb, nb, z, n_frames, max_iter, acc_bits;
 * int32 base[mb][nb]; uint8 syndromes[n_frames][ceil(m/8)];
 * int8 llr[n_frames][n].
 * Output file: uint8 bits[n_frames][ceil(n/8)]; uint8 converged[n_frames];
 * int32 iters[n_frames].
 * Exit status 0 on success; otherwise the failing call and ldpc_last_error()
 * (or the HIP error string) go to stderr.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "qkdldpc.h"

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));           \
            return 2;                                                                   \
        }                                                                               \
    } while (0)

#define LDPC_OK_OR_FAIL(call)                                                           \
    do {                                                                                \
        int r_ = (call);                                                                \
        if (r_ != LDPC_OK) {                                                            \
            fprintf(stderr, "%s returned %d: %s\n", #call, r_, ldpc_last_error());      \
            return 3;                                                                   \
        }                                                                               \
    } while (0)

static int read_exact(FILE *f, void *p, size_t n)
{
    return fread(p, 1, n, f) == n ? 0 : -1;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 1;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 1;
    }
    int32_t hdr[6];
    if (read_exact(in, hdr, sizeof hdr)) {
        fprintf(stderr, "short header\n");
        return 1;
    }
    const int32_t mb = hdr[0], nb = hdr[1], z = hdr[2], F = hdr[3], max_iter = hdr[4], acc_bits = hdr[5];
    if (mb < 1 || nb < 1 || z < 1 || F < 1 || (int64_t)nb * z >= (1LL << 31)) {
        fprintf(stderr, "bad header\n");
        return 1;
    }
    const size_t n = (size_t)nb * z, m = (size_t)mb * z;
    const size_t sb = (m + 7) / 8, bb = (n + 7) / 8;
    int32_t *base = malloc(sizeof(int32_t) * (size_t)mb * nb);
    uint8_t *h_syn = malloc(sb * F);
    int8_t *h_llr = malloc(n * F);
    uint8_t *h_bits = malloc(bb * F), *h_conv = malloc((size_t)F);
    int32_t *h_iters = malloc(sizeof(int32_t) * F);
    if (!base || !h_syn || !h_llr || !h_bits || !h_conv || !h_iters) {
        fprintf(stderr, "host allocation failed\n");
        return 1;
    }
    if (read_exact(in, base, sizeof(int32_t) * (size_t)mb * nb) || read_exact(in, h_syn, sb * F) ||
        read_exact(in, h_llr, n * F)) {
        fprintf(stderr, "short input\n");
        return 1;
    }
    fclose(in);

    ldpc_params prm;
    memset(&prm, 0, sizeof prm);  /* the paper's decoder */
    prm.acc_bits = acc_bits;
    ldpc_code *code = NULL;
    LDPC_OK_OR_FAIL(ldpc_code_create(base, mb, nb, z, &prm, &code));
    int32_t cn = 0, cm = 0;
    LDPC_OK_OR_FAIL(ldpc_code_dims(code, &cn, &cm, NULL, NULL, NULL));
    if ((size_t)cn != n || (size_t)cm != m) {
        fprintf(stderr, "ldpc_code_dims: n = %d, m = %d\n", cn, cm);
        return 1;
    }

    uint8_t *d_syn = NULL, *d_bits = NULL, *d_conv = NULL;
    int8_t *d_llr = NULL;
    int32_t *d_iters = NULL;
    void *d_ws = NULL;
    const size_t ws = ldpc_workspace_bytes(code, F);
    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));
    HIP_OK(hipMalloc((void **)&d_syn, sb * F));
    HIP_OK(hipMalloc((void **)&d_llr, n * F));
    HIP_OK(hipMalloc((void **)&d_bits, bb * F));
    HIP_OK(hipMalloc((void **)&d_conv, (size_t)F));
    HIP_OK(hipMalloc((void **)&d_iters, sizeof(int32_t) * F));
    if (ws)
        HIP_OK(hipMalloc(&d_ws, ws));
    HIP_OK(hipMemcpyAsync(d_syn, h_syn, sb * F, hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_llr, h_llr, n * F, hipMemcpyHostToDevice, stream));
    LDPC_OK_OR_FAIL(ldpc_decode_batch_ex(code, d_syn, d_llr, F, max_iter, d_bits, d_conv, d_iters, NULL, NULL,
                                         d_ws, ws, (void *)stream));
    HIP_OK(hipMemcpyAsync(h_bits, d_bits, bb * F, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(h_conv, d_conv, (size_t)F, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(h_iters, d_iters, sizeof(int32_t) * F, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));

    FILE *out = fopen(argv[2], "wb");
    if (!out) {
        perror(argv[2]);
        return 1;
    }
    if (fwrite(h_bits, 1, bb * F, out) != bb * F || fwrite(h_conv, 1, (size_t)F, out) != (size_t)F ||
        fwrite(h_iters, sizeof(int32_t), (size_t)F, out) != (size_t)F) {
        fprintf(stderr, "write failed\n");
        return 1;
    }
    fclose(out);

    int conv = 0;
    for (int32_t f = 0; f < F; ++f)
        conv += h_conv[f] != 0;
    printf("decoded %d frames of n = %zu: %d converged\n", F, n, conv);

    hipFree(d_syn);
    hipFree(d_llr);
    hipFree(d_bits);
    hipFree(d_conv);
    hipFree(d_iters);
    if (d_ws)
        hipFree(d_ws);
    HIP_OK(hipStreamDestroy(stream));
    ldpc_code_destroy(code);
    free(base);
    free(h_syn);
    free(h_llr);
    free(h_bits);
    free(h_conv);
    free(h_iters);
    return 0;
}
