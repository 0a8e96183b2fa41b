/* Host sanitizer run of the oracle: every entry point on seeded inputs,
 * including the error paths.  Built by tests/test_oracle_sanitized.py with
 * -fsanitize=address,undefined; any report makes the run fail. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "grand_oracle.h"

static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

/* H for a small code: rows x N, any 0/1 rows (the oracle only needs a matrix). */
static void random_h(uint32_t N, uint32_t rows, uint64_t *h)
{
    const uint32_t w = (N + 63) / 64;
    memset(h, 0, sizeof(uint64_t) * rows * w);
    for (uint32_t i = 0; i < rows; i++)
        for (uint32_t j = 0; j < N; j++)
            if (unif() < 0.5 || j == i)
                h[i * w + j / 64] |= 1ull << (j % 64);
}

int main(void)
{
    static const uint32_t Ns[] = {4, 8, 16, 32, 64, 128};
    static const uint32_t Ms[] = {4, 16, 64, 256};
    int fails = 0;
    for (unsigned a = 0; a < sizeof(Ns) / sizeof(Ns[0]); a++)
        for (unsigned b = 0; b < sizeof(Ms) / sizeof(Ms[0]); b++) {
            const uint32_t N = Ns[a], M = Ms[b], rows = N / 2;
            uint32_t m = 0;
            while ((1u << (2 * (m + 1))) <= M)
                m++;
            const uint32_t L = (N + 2 * m - 1) / (2 * m);
            float *rx = malloc(sizeof(float) * 2 * L);
            uint64_t *h = malloc(sizeof(uint64_t) * rows * ((N + 63) / 64));
            uint64_t cw[16];
            uint64_t q = 0;
            uint8_t ab = 0;
            random_h(N, rows, h);
            for (int trial = 0; trial < 8; trial++) {
                const int levels = 1 << m;
                for (uint32_t i = 0; i < 2 * L; i++) {
                    int lv = (int)(unif() * levels);
                    rx[i] = (float)(2 * lv - (levels - 1)) + (float)(unif() * 2.4 - 1.2);
                }
                if (trial == 7)
                    rx[0] = 4.0f * (float)levels;   /* far outside the constellation */
                if (orc_decode(N, rows, h, rx, M, 0.5, 200, cw, &q, &ab) != ORC_OK)
                    fails++;
                if (q < 1 || q > 200)
                    fails++;
                /* Algorithm 2's cut-off: selection and the restricted decode */
                uint8_t sel[512];
                uint32_t nsel = 0;
                const uint32_t S = 1 + (uint32_t)trial % 4;
                if (orc_select_symbols(N, M, rx, S, sel, &nsel) != ORC_OK || nsel != (S < L ? S : L))
                    fails++;
                if (orc_decode_ex(N, rows, h, rx, M, 0.5, 1u << 20, S, cw, &q, &ab) != ORC_OK ||
                    q < 1 || q > (1ull << (2 * S)))
                    fails++;
            }
            if (orc_select_symbols(N, M, rx, 0, NULL, NULL) == ORC_OK)
                fails++;
            /* error paths */
            if (orc_decode(N, rows, h, rx, 8, 0.5, 10, cw, &q, &ab) == ORC_OK)
                fails++;
            if (orc_decode(N, rows, h, rx, M, 0.5, 0, cw, &q, &ab) == ORC_OK)
                fails++;
            rx[0] = NAN;
            if (orc_decode(N, rows, h, rx, M, 0.5, 10, cw, &q, &ab) == ORC_OK)
                fails++;
            free(rx);
            free(h);
        }
    /* enumeration, including exhaustion of all 2^n patterns */
    uint32_t cs[12];
    for (int i = 0; i < 12; i++)
        cs[i] = (uint32_t)(i * 3 / 2);
    uint64_t masks[5000], costs[5000];
    if (orc_enumerate(12, cs, 5000, masks, costs) != 4096)
        fails++;
    /* Algorithm 1 on a dense matrix */
    uint8_t H[8 * 16], c[16], r[8];
    for (int i = 0; i < 8 * 16; i++)
        H[i] = unif() < 0.5;
    for (int i = 0; i < 16; i++)
        c[i] = unif() < 0.5;
    uint32_t steps = 0;
    uint64_t ands = 0, xors = 0;
    if (orc_pmult(8, 16, H, c, r, &steps, &ands, &xors) != ORC_OK)
        fails++;
    printf("oracle sanitizer run: %d failures\n", fails);
    return fails != 0;
}
