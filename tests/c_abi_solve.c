/* A plain C caller of the library: reads a CSR batch of 2D LPs from a binary
 * file, solves it on the GPU through rgb_solve_batch and rgb_solve_batch_noalloc
 * (device buffers from HIP's C runtime API, one non-blocking stream), and
 * writes x, y and status of both solves to a binary file.
 *
 * Input file: int64 num_lps, int64 num_constraints, int64 offsets[num_lps+1],
 * float ax[N], ay[N], b[N], cx[B], cy[B].  Output file: for each of the two
 * solves, float x[B], float y[B], int32 status[B].
 *
 * Usage: c_abi_solve IN OUT [variant]   (variant as rgb_variant_t, default AUTO)
 * Exit status 0 on success; a message on stderr otherwise. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "rgb.h"

#define CHECK_HIP(call)                                                   \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_)); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static int read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes ? 0 : -1; }

int main(int argc, char** argv) {
    if (argc < 3) {
        fprintf(stderr, "usage: %s IN OUT [variant]\n", argv[0]);
        return 2;
    }
    FILE* in = fopen(argv[1], "rb");
    if (!in) {
        fprintf(stderr, "cannot open %s\n", argv[1]);
        return 1;
    }
    int64_t B = 0, N = 0;
    if (read_all(in, &B, 8) || read_all(in, &N, 8) || B < 0 || N < 0) {
        fprintf(stderr, "bad header\n");
        return 1;
    }
    const size_t nb = (size_t)B, nn = (size_t)N;
    int64_t* offsets = malloc(8 * (nb + 1));
    float* rows = malloc(4 * (3 * nn + 2 * nb) + 4);
    if (!offsets || !rows || read_all(in, offsets, 8 * (nb + 1)) || read_all(in, rows, 4 * (3 * nn + 2 * nb))) {
        fprintf(stderr, "short input\n");
        return 1;
    }
    fclose(in);

    rgb_ctx_t* ctx = NULL;
    if (rgb_ctx_create(0, NULL, &ctx) != RGB_OK) {
        fprintf(stderr, "rgb_ctx_create failed\n");
        return 1;
    }
    hipStream_t stream;
    CHECK_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    int64_t* d_off = NULL;
    float *d_rows = NULL, *d_out = NULL;
    CHECK_HIP(hipMalloc((void**)&d_off, 8 * (nb + 1)));
    CHECK_HIP(hipMalloc((void**)&d_rows, 4 * (3 * nn + 2 * nb) + 4));
    CHECK_HIP(hipMalloc((void**)&d_out, 4 * 3 * nb + 4));
    CHECK_HIP(hipMemcpyAsync(d_off, offsets, 8 * (nb + 1), hipMemcpyHostToDevice, stream));
    CHECK_HIP(hipMemcpyAsync(d_rows, rows, 4 * (3 * nn + 2 * nb), hipMemcpyHostToDevice, stream));
    const float* ax = d_rows;
    const float* ay = d_rows + nn;
    const float* b = d_rows + 2 * nn;
    const float* cx = d_rows + 3 * nn;
    const float* cy = d_rows + 3 * nn + nb;
    float* x = d_out;
    float* y = d_out + nb;
    int32_t* st = (int32_t*)(d_out + 2 * nb);

    rgb_solve_opts_t opts = {0};
    opts.variant = argc > 3 ? atoi(argv[3]) : RGB_VARIANT_AUTO;
    float* host = malloc(4 * 3 * nb + 4);
    FILE* out = fopen(argv[2], "wb");
    if (!host || !out) {
        fprintf(stderr, "cannot write %s\n", argv[2]);
        return 1;
    }
    for (int pass = 0; pass < 2; ++pass) {
        rgb_err_t rc = pass == 0 ? rgb_solve_batch(ctx, B, N, d_off, ax, ay, b, cx, cy, x, y, st, &opts, stream)
                                 : rgb_solve_batch_noalloc(ctx, B, N, d_off, ax, ay, b, cx, cy, x, y, st, &opts,
                                                           stream);
        if (rc != RGB_OK) {
            fprintf(stderr, "solve %d failed (%d): %s\n", pass, (int)rc, rgb_ctx_last_error(ctx));
            return 1;
        }
        CHECK_HIP(hipMemcpyAsync(host, d_out, 4 * 3 * nb, hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        if (fwrite(host, 1, 4 * 3 * nb, out) != 4 * 3 * nb) {
            fprintf(stderr, "short write\n");
            return 1;
        }
        CHECK_HIP(hipMemsetAsync(d_out, 0, 4 * 3 * nb, stream));
    }
    fclose(out);
    CHECK_HIP(hipStreamSynchronize(stream));
    CHECK_HIP(hipFree(d_off));
    CHECK_HIP(hipFree(d_rows));
    CHECK_HIP(hipFree(d_out));
    CHECK_HIP(hipStreamDestroy(stream));
    rgb_ctx_destroy(ctx);
    free(host);
    free(rows);
    free(offsets);
    printf("solved %lld LPs twice\n", (long long)B);
    return 0;
}
