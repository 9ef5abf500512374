/* Plain C11 client of include/sfac.h: host-only entry points (no device work), so it runs
 * without a GPU. Exit status 0 when every check holds; prints the failing check otherwise. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sfac.h"

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(void) {
    /* axis tables of N = 63, alpha = 1.5: the diagonal method's length is N, the embedded
     * method's the power of two M >= 2N - 1 */
    int32_t len = 0, rad[12], nst = 0;
    CHECK(sfac_axis_tables(63, 1.5, 0.1, 0.01, 2.0 / 64, SFAC_METHOD_DIAG, &len, NULL, NULL, rad, &nst) == SFAC_OK);
    CHECK(len == 63 && nst >= 1);
    int32_t prod = 1;
    for (int i = 0; i < nst; ++i) prod *= rad[i];
    CHECK(prod == 63);
    CHECK(sfac_axis_tables(63, 1.5, 0.1, 0.01, 2.0 / 64, SFAC_METHOD_EMBED, &len, NULL, NULL, NULL, NULL) == SFAC_OK);
    CHECK(len == 128);
    double sc[63], ss[63];
    CHECK(sfac_axis_tables(63, 1.5, 0.1, 0.01, 2.0 / 64, SFAC_METHOD_DIAG, &len, sc, ss, NULL, NULL) == SFAC_OK);
    /* B is negative semi-definite, so every factor e^{t lambda}/N lies in (0, 1/N] */
    for (int j = 0; j < 63; ++j) CHECK(sc[j] > 0.0 && sc[j] <= 1.0 / 63 + 1e-15 && ss[j] > 0.0 && ss[j] <= 1.0 / 63 + 1e-15);

    /* argument validation happens before any device call */
    sfac_plan p = (sfac_plan)0x1;
    int32_t n[2] = {8, 8};
    double alpha[2] = {1.5, 1.5}, h[2] = {0.1, 0.1};
    CHECK(sfac_plan_create(&p, 4, n, alpha, 0.1, 0.01, h, SFAC_FP64, NULL, NULL) == SFAC_EINVAL);
    CHECK(p == NULL);
    CHECK(strstr(sfac_last_error(), "dims") != NULL);
    double bad_alpha[2] = {1.5, 2.5};
    CHECK(sfac_plan_create(&p, 2, n, bad_alpha, 0.1, 0.01, h, SFAC_FP64, NULL, NULL) == SFAC_EINVAL);
    sfac_options opt;
    memset(&opt, 0, sizeof opt);
    opt.method[0] = SFAC_METHOD_DIAG;
    int32_t prime[2] = {127, 8};
    CHECK(sfac_plan_create(&p, 2, prime, alpha, 0.1, 0.01, h, SFAC_FP64, NULL, &opt) == SFAC_EUNSUPPORTED);

    /* the exact exponential of one axis (host only): symmetric, entries in (-1, 1], rows of a
     * contraction (B is negative definite); the exact method asks for every axis and FP64 */
    static double P[31 * 31];
    CHECK(sfac_exact_exponential(31, 1.7, 0.1, 0.05, 2.0 / 32, P) == SFAC_OK);
    for (int i = 0; i < 31; ++i) {
        double row = 0.0;
        for (int j = 0; j < 31; ++j) {
            CHECK(P[i * 31 + j] == P[j * 31 + i]);
            row += fabs(P[i * 31 + j]);
        }
        CHECK(P[i * 31 + i] > 0.0 && P[i * 31 + i] <= 1.0);
        CHECK(row > 0.0 && row <= sqrt(31.0));
    }
    CHECK(sfac_exact_exponential(1025, 1.5, 0.1, 0.01, 2.0 / 1026, P) == SFAC_EUNSUPPORTED);
    CHECK(sfac_exact_exponential(31, 1.5, 0.1, 0.01, 2.0 / 32, NULL) == SFAC_EINVAL);
    memset(&opt, 0, sizeof opt);
    opt.method[0] = SFAC_METHOD_EXACT;
    CHECK(sfac_plan_create(&p, 2, n, alpha, 0.1, 0.01, h, SFAC_FP64, NULL, &opt) == SFAC_EINVAL);
    opt.method[1] = SFAC_METHOD_EXACT;
    CHECK(sfac_plan_create(&p, 2, n, alpha, 0.1, 0.01, h, SFAC_FP32, NULL, &opt) == SFAC_EUNSUPPORTED);

    /* NULL handles */
    CHECK(sfac_step(NULL, NULL, 1) == SFAC_EINVAL);
    CHECK(sfac_plan_destroy(NULL) == SFAC_OK);
    CHECK(sfac_plan_device_bytes(NULL) == 0);
    CHECK(sfac_batch_destroy(NULL) == SFAC_OK);
    CHECK(sfac_group_destroy(NULL) == SFAC_OK);
    printf("c abi host calls: ok\n");
    return 0;
}
