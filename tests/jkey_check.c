/* Host check of the selection key of the GPU local-KNN kernel (k_knn.hip).
 *
 * The kernel ranks candidates by key(I, U) = floor(I * (2^32 - 1) / U) and
 * later recovers I from the key and S = |P_u| + |P_v|.  Both are computed in
 * fp32 around the hardware reciprocal (v_rcp_f32, within 1 ulp), so this
 * program restates the kernel's two functions in C, feeds them reciprocals
 * that are correctly rounded or off by up to `ulps` ulps, and compares with
 * exact integer arithmetic over every pair the kernel can see: profiles of
 * fewer than 2^15 items, so S <= 65534, U = S - I and 0 <= I <= S / 2.
 *
 * Usage: jkey_check ULPS STRIDE   (checks every STRIDE-th union size U;
 * prints the number of mismatches of each function, exits 1 on any). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static float rcp_off(float x, int d)
{
    float r = 1.0f / x;
    for (; d > 0; --d) r = nextafterf(r, INFINITY);
    for (; d < 0; ++d) r = nextafterf(r, 0.0f);
    return r;
}

/* the kernel's jkey(), with its reciprocal r of U given */
static uint32_t jkey_host(uint32_t I, uint32_t U, float r)
{
    const float qf = (float)I * r * 4294967296.0f;
    const uint32_t q0 = qf >= 4294967295.0f ? 0xFFFFFFFFu : (uint32_t)qf;
    const int32_t rem = (int32_t)((0u - I) - q0 * U);
    const int32_t c = (int32_t)floorf((float)rem * r);
    uint32_t q = q0 + (uint32_t)c;
    const int32_t rem1 = rem - c * (int32_t)U;
    if (rem1 < 0) q -= 1;
    else if (rem1 >= (int32_t)U) q += 1;
    return q;
}

/* the kernel's key_to_I(), with its reciprocal r of 2^32 - 1 + key given;
 * fused: the final rounding add contracted into a fused multiply-add */
static uint32_t key_to_I_host(uint32_t key, uint32_t S, float r, int fused)
{
    const float kt = (float)key;
    const float sk = (float)S * kt;
    const float x = fused ? fmaf(sk, r, 0.5f) : sk * r + 0.5f;
    return (uint32_t)x;
}

int main(int argc, char **argv)
{
    const int ulps = argc > 1 ? atoi(argv[1]) : 0;
    const int stride = argc > 2 ? atoi(argv[2]) : 1;
    const uint32_t smax = 65534;
    unsigned long long bad_key = 0, bad_i = 0, pairs = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad_key, bad_i, pairs)
    for (int64_t Ui = 1; Ui <= (int64_t)smax; Ui += stride) {
        const uint32_t U = (uint32_t)Ui;
        /* exact floor(I * (2^32 - 1) / U), stepped in I without division */
        const uint64_t num = 0xFFFFFFFFull;
        const uint64_t dq = num / U, dr = num % U;
        uint64_t q = 0, rr = 0;
        const uint32_t imax = U < smax - U ? U : smax - U;  /* I <= U and I + U <= smax */
        for (uint32_t I = 0; I <= imax; ++I) {
            for (int d = -ulps; d <= ulps; ++d) {
                const uint32_t k = jkey_host(I, U, rcp_off((float)U, d));
                bad_key += k != (uint32_t)q;
                /* recovery from the exact key */
                const float kt = (float)(uint32_t)q;
                const float r2 = rcp_off(4294967295.0f + kt, d);
                bad_i += key_to_I_host((uint32_t)q, I + U, r2, 0) != I;
                bad_i += key_to_I_host((uint32_t)q, I + U, r2, 1) != I;
            }
            ++pairs;
            q += dq;
            rr += dr;
            if (rr >= U) { rr -= U; ++q; }
        }
    }
    printf("pairs %llu ulps %d: key mismatches %llu, I mismatches %llu\n", pairs, ulps, bad_key,
           bad_i);
    return bad_key || bad_i ? 1 : 0;
}
