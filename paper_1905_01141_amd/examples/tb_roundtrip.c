/*
 * tb_roundtrip.c -- the C ABI of libtdec used from plain C (no Python, no
 * torch): encode a transport block on the GPU, map the coded bits to
 * noiseless int16 LLRs, decode it, and check that the payload comes back and
 * CRC24A passes.  Exit status 0 on success.
 *
 *   usage: tb_roundtrip [tbs]   (default 75376 bits: 13 code blocks of K=5824)
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tdec.h"

#define CHECK_HIP(x)                                                          \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));    \
            return 2;                                                         \
        }                                                                     \
    } while (0)
#define CHECK_TDEC(x)                                                         \
    do {                                                                      \
        tdec_status s_ = (x);                                                 \
        if (s_ != TDEC_OK) {                                                  \
            fprintf(stderr, "%s failed: %d\n", #x, (int)s_);                  \
            return 3;                                                         \
        }                                                                     \
    } while (0)

int main(int argc, char **argv)
{
    const int32_t tbs = argc > 1 ? atoi(argv[1]) : 75376;
    const int64_t n_llr = tdec_tb_llr_count(tbs);
    if (n_llr < 0) {
        fprintf(stderr, "tbs %d out of range\n", tbs);
        return 1;
    }
    tdec_seg seg;
    CHECK_TDEC(tdec_segment(tbs, &seg));
    const size_t nbytes = ((size_t)tbs + 7) / 8;

    /* random payload, packed MSB first */
    uint8_t *pay = (uint8_t *)malloc(nbytes);
    uint32_t x = 12345u;
    for (size_t i = 0; i < nbytes; ++i) {
        x = x * 1664525u + 1013904223u;
        pay[i] = (uint8_t)(x >> 24);
    }
    if (tbs % 8) pay[nbytes - 1] &= (uint8_t)(0xFFu << (8 - tbs % 8));

    tdec_ctx *ctx = NULL;
    CHECK_TDEC(tdec_create(0, 0, &ctx));
    uint8_t *d_pay, *d_coded, *d_bits;
    int16_t *d_llr;
    tdec_tb_result *d_res;
    CHECK_HIP(hipMalloc((void **)&d_pay, nbytes));
    CHECK_HIP(hipMalloc((void **)&d_coded, (size_t)n_llr));
    CHECK_HIP(hipMalloc((void **)&d_llr, (size_t)n_llr * sizeof(int16_t)));
    CHECK_HIP(hipMalloc((void **)&d_bits, nbytes));
    CHECK_HIP(hipMalloc((void **)&d_res, sizeof(tdec_tb_result)));
    CHECK_HIP(hipMemcpy(d_pay, pay, nbytes, hipMemcpyHostToDevice));

    /* encode on the GPU, then noiseless LLRs: bit 1 -> +400, bit 0 -> -400 */
    CHECK_TDEC(tb_encode(ctx, d_pay, tbs, d_coded, NULL));
    uint8_t *coded = (uint8_t *)malloc((size_t)n_llr);
    int16_t *llr = (int16_t *)malloc((size_t)n_llr * sizeof(int16_t));
    CHECK_HIP(hipMemcpy(coded, d_coded, (size_t)n_llr, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n_llr; ++i) llr[i] = coded[i] ? 400 : -400;
    CHECK_HIP(hipMemcpy(d_llr, llr, (size_t)n_llr * sizeof(int16_t), hipMemcpyHostToDevice));

    /* decode: up to 8 iterations with CRC stop, the library's window count */
    const tdec_params p = {8, TDEC_STOP_CRC, 0, 1, 0};
    CHECK_HIP(hipMemset(d_bits, 0, nbytes));
    CHECK_TDEC(tb_decode(ctx, d_llr, tbs, &p, d_bits, d_res, NULL));
    CHECK_HIP(hipDeviceSynchronize());

    uint8_t *bits = (uint8_t *)malloc(nbytes);
    tdec_tb_result res;
    CHECK_HIP(hipMemcpy(bits, d_bits, nbytes, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(&res, d_res, sizeof res, hipMemcpyDeviceToHost));
    const int same = memcmp(bits, pay, nbytes) == 0;
    printf("tbs %d: C=%d K+=%d K-=%d F=%d; tb_ok=%d, iterations=%d, payload %s\n", tbs, seg.C,
           seg.Kplus, seg.Kminus, seg.F, res.tb_ok, res.max_iters_used,
           same ? "identical" : "DIFFERENT");

    tdec_destroy(ctx);
    hipFree(d_pay);
    hipFree(d_coded);
    hipFree(d_llr);
    hipFree(d_bits);
    hipFree(d_res);
    free(pay);
    free(coded);
    free(llr);
    free(bits);
    return (res.tb_ok == 1 && same) ? 0 : 4;
}
