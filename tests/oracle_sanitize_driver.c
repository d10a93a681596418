/* Test support: the oracle's C source built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (see tests/test_oracle_sanitize.py).  Runs key
 * generation and full-domain bootstraps of every message at the smallest
 * configuration (n=64 N=256 t=8) and checks each decrypts to its table entry;
 * prints "ok" and exits 0 on success. */
#include "../oracle/fdfb_oracle.c"

#include <stdio.h>

int main(void)
{
    const double q = 4294967296.0;
    or_params P = {64, 256, 3, 8, 2, 4, 4, 4, 4, 2, 2, q / 1048576.0, q / 268435456.0, q / 268435456.0,
                   q / 1048576.0};
    const uint32_t n = P.n, N = P.N, t = 1u << P.log2_t;
    uint32_t *s = calloc(n, 4), *sf = calloc(N, 4);
    uint32_t *brk = calloc((size_t)n * 2 * P.g_ell * 2 * N, 4);
    uint32_t *pk = calloc((size_t)N * P.pk_ell * 2 * N, 4);
    uint32_t *ksk = calloc((size_t)N * P.ks_ell * (n + 1), 4);
    int32_t *p0 = calloc(N, 4), *p1 = calloc(N, 4);
    uint32_t *ct = calloc(n + 1, 4), *out = calloc(N + 1, 4);
    if (!s || !sf || !brk || !pk || !ksk || !p0 || !p1 || !ct || !out) return 2;
    or_keygen(&P, 1001, s, sf, brk, pk, ksk);
    const uint32_t lut[8] = {3, 1, 4, 1, 5, 2, 6, 0};
    or_setup_polynomial(lut, t, N, p0, p1);
    int bad = 0;
    for (uint32_t m = 0; m < t; ++m) {
        or_encrypt(&P, s, m, 2001, m, ct);
        or_fdfb(&P, brk, pk, ksk, p0, p1, ct, 0, out, NULL);
        int64_t e = 0;
        const uint32_t got = or_decrypt(out, s, n, P.log2_t, &e);
        if (got != lut[m]) {
            printf("m=%u: got %u, want %u\n", m, got, lut[m]);
            bad = 1;
        }
    }
    free(s); free(sf); free(brk); free(pk); free(ksk); free(p0); free(p1); free(ct); free(out);
    if (bad) return 1;
    printf("ok\n");
    return 0;
}
