/*
 * Reference ("oracle") summation routines -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is a plain, deliberately simple CPU implementation of what the
 * device-wide sum reduction computes: the sum of the elements of an array
 * (the reduction case study, Section VII of Zhang, Wahib, Zhang, Matsuoka,
 * "A Study of Single and Multi-device Synchronization Methods in Nvidia
 * GPUs").  It is compiled with gcc, shares no code with the HIP library, and
 * may only be used by the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark.  The product path never links or calls it.
 *
 * Definitions implemented here (no blocking, fusion or reordering):
 *   - int32 input: S = sum_i x_i over the integers, accumulated in int64.
 *     Exact for every int32 input when n <= 2^32, because |S| <= 2^63.
 *   - fp32 / bf16 / fp16 input: S* = sum_i v(x_i) over the reals, where v()
 *     is the exact real value of each bit pattern.  Every finite value of
 *     these formats is an integer significand M times a power of two fixed by
 *     the biased exponent E, so S* is accumulated exactly as one int64 bin
 *     per biased exponent ("long accumulator"):
 *        fp32 (and bf16 = top 16 bits of an fp32):
 *            v = (-1)^s * M * 2^(max(E,1) - 150),  M = m + (E>0) * 2^23
 *        fp16:
 *            v = (-1)^s * M * 2^(max(E,1) - 25),   M = m + (E>0) * 2^10
 *     bins[E] += (-1)^s * M.  With M < 2^24 a bin cannot overflow int64 for
 *     n < 2^39.  The caller combines the bins with arbitrary-precision
 *     integers and rounds once (oracle.py).
 *   - A plain FP64 Neumaier-compensated sum, kept only as a secondary,
 *     independent cross-check of the exact result.
 *
 * NaN / infinity inputs are counted separately (they have no bin).
 */
#include <stdint.h>
#include <string.h>

/* Sum of int32 values in int64.  Returns the sum. */
int64_t oracle_sum_i32(const int32_t *x, int64_t n)
{
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i)
        s += (int64_t)x[i];
    return s;
}

/* Add one binary32 bit pattern into the exponent bins. */
static void bin_add_f32_bits(uint32_t b, int64_t bins[256], int64_t special[3])
{
    uint32_t sign = b >> 31;
    uint32_t e = (b >> 23) & 0xffu;
    uint32_t m = b & 0x7fffffu;
    if (e == 0xffu) {
        if (m != 0)
            special[0] += 1;          /* NaN */
        else if (sign)
            special[2] += 1;          /* -inf */
        else
            special[1] += 1;          /* +inf */
        return;
    }
    int64_t M = (int64_t)m + (e > 0 ? ((int64_t)1 << 23) : 0);
    bins[e] += sign ? -M : M;
}

/*
 * Exact exponent bins of n fp32 values.
 * bins: 256 int64 (caller-owned, overwritten); special: 3 int64 counts
 * {NaN, +inf, -inf} (caller-owned, overwritten).
 */
void oracle_bins_f32(const uint32_t *bits, int64_t n, int64_t *bins, int64_t *special)
{
    memset(bins, 0, 256 * sizeof(int64_t));
    memset(special, 0, 3 * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        bin_add_f32_bits(bits[i], bins, special);
}

/*
 * Exact exponent bins of n bfloat16 values.  A bfloat16 is the upper half
 * of a binary32, so its value is the binary32 with the low 16 bits zero.
 */
void oracle_bins_bf16(const uint16_t *bits, int64_t n, int64_t *bins, int64_t *special)
{
    memset(bins, 0, 256 * sizeof(int64_t));
    memset(special, 0, 3 * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        bin_add_f32_bits((uint32_t)bits[i] << 16, bins, special);
}

/*
 * Exact exponent bins of n binary16 values (bins has 32 entries used,
 * indexed by the 5-bit biased exponent).
 */
void oracle_bins_f16(const uint16_t *bits, int64_t n, int64_t *bins, int64_t *special)
{
    memset(bins, 0, 32 * sizeof(int64_t));
    memset(special, 0, 3 * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b = bits[i];
        uint32_t sign = b >> 15;
        uint32_t e = (b >> 10) & 0x1fu;
        uint32_t m = b & 0x3ffu;
        if (e == 0x1fu) {
            if (m != 0)
                special[0] += 1;
            else if (sign)
                special[2] += 1;
            else
                special[1] += 1;
            continue;
        }
        int64_t M = (int64_t)m + (e > 0 ? ((int64_t)1 << 10) : 0);
        bins[e] += sign ? -M : M;
    }
}

/*
 * Plain FP64 Neumaier (improved Kahan-Babuska) sum of values given as
 * doubles.  Secondary cross-check only; not exact.
 */
double oracle_neumaier_f64(const double *x, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + x[i];
        if ((s >= 0 ? s : -s) >= (x[i] >= 0 ? x[i] : -x[i]))
            c += (s - t) + x[i];
        else
            c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}
