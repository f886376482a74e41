/*
 * Oracle (test infrastructure only): schoolbook negacyclic polynomial
 * multiply-accumulate over Z[X]/(X^N + 1), reduced mod 2^32.
 *
 * The torus polynomials of §3.1 (T_N[X] = R[X]/(X^N+1) mod 1) are held as
 * Torus32 coefficients (value * 2^32 mod 2^32).  Multiplying an integer
 * polynomial u by a torus polynomial K is the textbook product with the
 * reduction X^N = -1:
 *
 *     (u * K)_m = sum_{p <= m} u_p K_{m-p}  -  sum_{p > m} u_p K_{N+m-p}
 *
 * computed here literally, in wrapping uint32 arithmetic.  No blocking,
 * reordering or transform: this is the definition written out.
 */
#include <stdint.h>

void oracle_negacyclic_mac(uint32_t *acc, const int32_t *u, const uint32_t *K,
                           int64_t N)
{
    for (int64_t p = 0; p < N; ++p) {
        const uint32_t up = (uint32_t)u[p];
        if (up == 0)
            continue;
        /* terms with p <= m: + u_p K_{m-p} */
        for (int64_t m = p; m < N; ++m)
            acc[m] += up * K[m - p];
        /* terms with p > m: X^{p+(N+m-p)} = X^{N+m} = -X^m */
        for (int64_t m = 0; m < p; ++m)
            acc[m] -= up * K[N + m - p];
    }
}
