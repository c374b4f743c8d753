/* Host check of the fp32 candidate filter of the GPU local-KNN kernel
 * (k_knn.hip, BeatTest).
 *
 * Once a row's heap is full, a candidate v can enter only if its key is at
 * least the root's key kt (a higher key, or the same key and a lower id).
 * With key(I, U) = floor(I * (2^32 - 1) / U) and U = S - I, S = |P_u| + |P_v|,
 * that holds exactly when I * (2^32 - 1 + kt) >= kt * S, i.e. for every I at
 * or above I* = ceil(kt * S / (2^32 - 1 + kt)).  The kernel turns a candidate
 * away when, in fp32,
 *     sigma = kt * rcp(2^32 - 1 + kt),  s = sigma * MARGIN,  sL = s * |P_u|,
 *     I < fma(s, |P_v|, sL)
 * (rcp: the hardware reciprocal, within 1 ulp).  The filter is safe if I*
 * always passes (the test does not depend on I otherwise, so every larger I
 * passes too).  This program restates the kernel's arithmetic in C, with the
 * reciprocal correctly rounded or off by up to `ulps` ulps (and, as a second
 * form, the quotient sigma itself so rounded or off), and checks I* against it
 * for a set of root keys, every STRIDE-th S up to 65534 (profiles below 2^15
 * items) and several splits of S into |P_u| + |P_v| with both at least I*.
 * It also checks the two exclusions the kernel folds into the same test: a
 * padded column has |P_v| = +inf and an inactive row s = NaN, and both fail
 * the comparison whatever s and I are.
 *
 * Usage: filter_check MARGIN ULPS STRIDE  (the kernel's margin is 0.999999;
 * prints the number of candidates wrongly turned away, exits 1 on any). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static float off_ulps(float x, int d)
{
    for (; d > 0; --d) x = nextafterf(x, INFINITY);
    for (; d < 0; ++d) x = nextafterf(x, 0.0f);
    return x;
}

/* exact floor(I * (2^32 - 1) / U) */
static uint32_t key_exact(uint32_t I, uint32_t U)
{
    return (uint32_t)((uint64_t)I * 0xFFFFFFFFull / U);
}

int main(int argc, char **argv)
{
    const float margin = argc > 1 ? (float)atof(argv[1]) : 0.999999f;
    const int ulps = argc > 2 ? atoi(argv[2]) : 0;
    const int stride = argc > 3 ? atoi(argv[3]) : 1;
    const uint32_t smax = 65534;
    /* root keys: the edges, keys of the closest fractions, and keys of
     * pseudo-random pairs (I, U) with U < 2^16 (a 64-bit LCG) */
    enum { NR = 640 };
    uint32_t roots[NR];
    int nr = 0;
    roots[nr++] = 1;
    roots[nr++] = key_exact(1, 65534);
    roots[nr++] = key_exact(1, 2);
    roots[nr++] = key_exact(32766, 32768);
    roots[nr++] = key_exact(65533, 65534);
    roots[nr++] = 0xFFFFFFFFu;
    uint64_t st = 0x9E3779B97F4A7C15ull;
    while (nr < NR) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        const uint32_t U = 1 + (uint32_t)((st >> 33) % 65534);
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        const uint32_t I = (uint32_t)((st >> 33) % (U + 1));
        const uint32_t k = key_exact(I, U);
        if (k > 0) roots[nr++] = k;
    }
    unsigned long long bad = 0, checked = 0;
    /* the exclusions: +inf length (padded column), NaN slope (inactive row) */
    {
        const float I_max = 65535.0f, svals[3] = {0.0f, 1e-9f, 0.5f};
        for (int q = 0; q < 3; ++q) {
            bad += I_max >= fmaf(svals[q], INFINITY, svals[q] * 100.0f);
            bad += I_max >= fmaf(NAN, 100.0f, NAN * 100.0f);
        }
    }
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : bad, checked)
    for (int ri = 0; ri < nr; ++ri) {
        const uint32_t kt = roots[ri];
        const uint64_t den = 0xFFFFFFFFull + kt;
        for (int form = 0; form < 2; ++form)
        for (int d = -ulps; d <= ulps; ++d) {
            const float ktf = (float)kt;
            const float den_f = 4294967295.0f + ktf;
            const float sigma = form ? ktf * off_ulps(1.0f / den_f, d) : off_ulps(ktf / den_f, d);
            const float s = sigma * margin;
            for (uint32_t S = 1; S <= smax; S += (uint32_t)stride) {
                const uint64_t Istar = ((uint64_t)kt * S + den - 1) / den;
                if (2 * Istar > S) continue; /* I <= min(|P_u|, |P_v|) */
                /* sanity of I*: it reaches the root's key, I* - 1 does not */
                if (key_exact((uint32_t)Istar, S - (uint32_t)Istar) < kt ||
                    (Istar > 0 && key_exact((uint32_t)Istar - 1, S - (uint32_t)Istar + 1) >= kt)) {
                    ++bad;
                    continue;
                }
                const uint32_t lo = (uint32_t)Istar, hi = S - (uint32_t)Istar;
                const uint32_t splits[5] = {lo, hi, S / 2, lo + (hi - lo) / 3, hi - (hi - lo) / 7};
                for (int q = 0; q < 5; ++q) {
                    const uint32_t Lu = splits[q], Lv = S - Lu;
                    const float sL = s * (float)Lu;
                    const float thr = fmaf(s, (float)Lv, sL);
                    bad += (float)Istar < thr;
                    ++checked;
                }
            }
        }
    }
    printf("roots %d ulps %d checked %llu: turned away %llu\n", nr, ulps, checked, bad);
    return bad ? 1 : 0;
}
