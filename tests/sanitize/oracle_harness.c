/*
 * Host harness of the oracle's C routines (oracle/oracle_sum.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by the test suite.  Every
 * routine runs over empty, single-element, special-value and random inputs,
 * with each buffer allocated at exactly its size so an access past its end
 * is reported, and each result is checked against a plain definition.
 * Exit status 0 when every check holds (a sanitizer report aborts).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_sum_i32(const int32_t *x, int64_t n);
void oracle_bins_f32(const uint32_t *bits, int64_t n, int64_t *bins, int64_t *special);
void oracle_bins_bf16(const uint16_t *bits, int64_t n, int64_t *bins, int64_t *special);
void oracle_bins_f16(const uint16_t *bits, int64_t n, int64_t *bins, int64_t *special);
double oracle_neumaier_f64(const double *x, int64_t n);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

/* value of the fp32 bins as a long double (exact for these small cases) */
static long double bins_value_f32(const int64_t *bins) {
    long double v = 0;
    for (int e = 0; e < 255; ++e)
        v += ldexpl((long double)bins[e], (e > 0 ? e : 1) - 150);
    return v;
}

int main(void) {
    int64_t *bins = malloc(256 * sizeof(int64_t));
    int64_t *special = malloc(3 * sizeof(int64_t));
    for (int64_t n = 0; n <= 4099; n += (n < 10 ? 1 : 409)) {
        /* int32: extremes and random values, against a plain loop */
        int32_t *xi = malloc((size_t)(n ? n : 1) * sizeof(int32_t));
        int64_t want = 0;
        for (int64_t i = 0; i < n; ++i) {
            xi[i] = (i % 3 == 0) ? INT32_MIN : (i % 3 == 1) ? INT32_MAX : (int32_t)(rnd() & 0xFFFFFFFFu);
            want += xi[i];
        }
        CHECK(oracle_sum_i32(xi, n) == want);
        free(xi);
        /* fp32 bit patterns: small integers (exact in long double) plus
         * specials, against a direct sum */
        uint32_t *xf = malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
        long double wantf = 0;
        int64_t nan = 0, pinf = 0, ninf = 0;
        for (int64_t i = 0; i < n; ++i) {
            float v = (float)((int)(rnd() % 2001) - 1000) * 0.25f;
            uint32_t b;
            memcpy(&b, &v, 4);
            if (i % 97 == 5) { b = 0x7fc00000u; ++nan; }
            else if (i % 101 == 7) { b = 0x7f800000u; ++pinf; }
            else if (i % 103 == 9) { b = 0xff800000u; ++ninf; }
            else if (i % 89 == 3) { b = 0x00000001u; v = ldexpf(1.0f, -149); wantf += v; }
            else wantf += v;
            xf[i] = b;
        }
        oracle_bins_f32(xf, n, bins, special);
        CHECK(special[0] == nan && special[1] == pinf && special[2] == ninf);
        CHECK(bins_value_f32(bins) == wantf);
        /* bf16: the top halves of the same patterns */
        uint16_t *xb = malloc((size_t)(n ? n : 1) * sizeof(uint16_t));
        for (int64_t i = 0; i < n; ++i) xb[i] = (uint16_t)(xf[i] >> 16);
        oracle_bins_bf16(xb, n, bins, special);
        CHECK(special[0] + special[1] + special[2] <= n);
        free(xb);
        free(xf);
        /* fp16: every exponent, both signs */
        uint16_t *xh = malloc((size_t)(n ? n : 1) * sizeof(uint16_t));
        int64_t wanth_units = 0; /* in units of 2^-24 for finite values below 2^15 */
        for (int64_t i = 0; i < n; ++i) {
            uint16_t b = (uint16_t)(rnd() & 0x7BFFu); /* finite, below the top exponent */
            if (rnd() & 1) b |= 0x8000u;
            xh[i] = b;
            int e = (b >> 10) & 0x1f, m = b & 0x3ff;
            int64_t M = m + (e > 0 ? 1024 : 0);
            int64_t units = M << ((e > 0 ? e : 1) - 1);
            wanth_units += (b & 0x8000u) ? -units : units;
        }
        oracle_bins_f16(xh, n, bins, special);
        int64_t got_units = 0;
        for (int e = 0; e < 31; ++e) got_units += bins[e] * ((int64_t)1 << ((e > 0 ? e : 1) - 1));
        CHECK(got_units == wanth_units);
        free(xh);
        /* Neumaier on doubles whose exact sum is representable */
        double *xd = malloc((size_t)(n ? n : 1) * sizeof(double));
        double wantd = 0;
        for (int64_t i = 0; i < n; ++i) {
            xd[i] = (double)((int64_t)(rnd() % 2000001) - 1000000);
            wantd += xd[i];
        }
        CHECK(oracle_neumaier_f64(xd, n) == wantd);
        free(xd);
    }
    free(bins);
    free(special);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle harness ok\n");
    return 0;
}
