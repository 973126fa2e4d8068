/*
 * General lagged-Fibonacci oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain CPU implementation of the combined generator of Haramoto & Suzuki
 * (arXiv 2512.00093), Sec. 2, for arbitrary parameters: lags (r, s) with
 * 1 <= s < r, precision e (words in Z/2^e, 1 <= e <= 32) and the arithmetic
 * sequence c_n = c_{n-1} - d mod m with M = 2^e, 1 <= m <= 2^e - 1 (or any
 * m >= 1 when e = 32), d < m.  RANMAR is the case (97, 33, 24, 2^24 - 3,
 * 7654321).  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code with the RANMAR oracle beside it nor
 * with the GPU library.
 *
 * Contents, each following the passage it cites:
 *   - literal J-fold stepping of f = (f_1, f_2)    (Sec. 2, f^J)
 *   - draws: step, then output (x - c) mod 2^e     (Sec. 2 output; Algorithm 2)
 *   - t^J mod phi(t), phi = t^r + t^{r-s} - 1,
 *     over Z/2^e by left-to-right binary powering:
 *     schoolbook square, then long division by
 *     the monic phi; a set bit multiplies by t     (Sec. 3.1, P_J; Sec. 5 cost
 *                                                   O(r^2 log J))
 *   - u P_J(A) by Horner's rule                     (Sec. 3.1, Horner formula)
 *   - c_J = (c - J d) mod m                         (Sec. 3.2)
 *
 * State record: r + 1 words, u_1 .. u_r (u_1 the oldest) then c, as in the
 * RANMAR oracle.  Every function assumes parameters that lfg_check accepts.
 * Parity status: pinned by the CPU tests (reduction to RANMAR and its paper
 * values, brute-force stepping, the closed forms of t^J for J <= r + s, and
 * the period 2^{e-1}(2^r - 1) of primitive trinomials).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint32_t emask(uint32_t e) { return e >= 32 ? 0xFFFFFFFFu : ((1u << e) - 1u); }

int lfg_check(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d)
{
    if (r < 2 || s < 1 || s >= r || e < 1 || e > 32) return -1;
    if (m < 1 || (e < 32 && m > emask(e)) || d >= m) return -1;
    return 0;
}

/* f_1: (u_1, ..., u_r) -> (u_2, ..., u_r, u_1 - u_{r-s+1}). */
static void f1(uint32_t r, uint32_t s, uint32_t mask, uint32_t *u)
{
    uint32_t nw = (u[0] - u[r - s]) & mask;
    memmove(u, u + 1, (size_t)(r - 1) * sizeof(uint32_t));
    u[r - 1] = nw;
}

/* f_2: c -> c - d mod m. */
static uint32_t f2(uint32_t m, uint32_t d, uint32_t c)
{
    return c >= d ? c - d : (uint32_t)((uint64_t)c + m - d);
}

/* Literal f^J: J applications of the transition. */
void lfg_step(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d,
              const uint32_t *u_in, uint32_t c, uint64_t J, uint32_t *u_out, uint32_t *c_out)
{
    uint32_t mask = emask(e);
    uint32_t *u = (uint32_t *)malloc(r * sizeof(uint32_t));
    memcpy(u, u_in, r * sizeof(uint32_t));
    for (uint64_t q = 0; q < J; ++q) {
        f1(r, s, mask, u);
        c = f2(m, d, c);
    }
    memcpy(u_out, u, r * sizeof(uint32_t));
    *c_out = c;
    free(u);
}

/* n draws: each steps (u, c) and outputs (newest word - c) mod 2^e. */
void lfg_draws(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d,
               const uint32_t *u_in, uint32_t c, uint64_t n, uint32_t *out,
               uint32_t *u_out, uint32_t *c_out)
{
    uint32_t mask = emask(e);
    uint32_t *u = (uint32_t *)malloc(r * sizeof(uint32_t));
    memcpy(u, u_in, r * sizeof(uint32_t));
    for (uint64_t q = 0; q < n; ++q) {
        f1(r, s, mask, u);
        c = f2(m, d, c);
        if (out) out[q] = (u[r - 1] - c) & mask;
    }
    if (u_out) memcpy(u_out, u, r * sizeof(uint32_t));
    if (c_out) *c_out = c;
    free(u);
}

/* Long division of prod (degree <= deg) by the monic phi = t^r + t^{r-s} - 1:
 * for k = deg .. r, subtract q t^{k-r} phi with q = prod[k]. */
static void reduce_phi(uint32_t r, uint32_t s, uint32_t mask, uint32_t *prod, uint32_t deg)
{
    for (uint32_t k = deg; k >= r; --k) {
        uint32_t q = prod[k];
        prod[k] = 0;                                           /* q t^k          */
        prod[k - s] = (prod[k - s] - q) & mask;                /* q t^{k-s}      */
        prod[k - r] = (prod[k - r] + q) & mask;                /* - q (-1) t^{k-r} */
    }
}

/* P_J(t) = t^J mod phi over Z/2^e, J = jhi 2^64 + jlo; P has r coefficients. */
void lfg_xpow(uint32_t r, uint32_t s, uint32_t e, uint64_t jlo, uint64_t jhi, uint32_t *P)
{
    uint32_t mask = emask(e);
    uint32_t *prod = (uint32_t *)calloc(2 * (size_t)r, sizeof(uint32_t));
    memset(P, 0, r * sizeof(uint32_t));
    P[0] = 1 & mask;
    int top = 127;  /* start at the highest set bit of J (squaring 1 is 1) */
    while (top >= 0 && !(top >= 64 ? (jhi >> (top - 64)) & 1 : (jlo >> top) & 1)) --top;
    for (int bit = top; bit >= 0; --bit) {
        /* square */
        memset(prod, 0, 2 * (size_t)r * sizeof(uint32_t));
        for (uint32_t i = 0; i < r; ++i)
            for (uint32_t j = 0; j < r; ++j)
                prod[i + j] = (prod[i + j] + P[i] * P[j]) & mask;
        reduce_phi(r, s, mask, prod, 2 * r - 2);
        memcpy(P, prod, r * sizeof(uint32_t));
        int set = bit >= 64 ? (int)((jhi >> (bit - 64)) & 1) : (int)((jlo >> bit) & 1);
        if (set) {
            /* multiply by t: shift up one place, then reduce the t^r term */
            memset(prod, 0, 2 * (size_t)r * sizeof(uint32_t));
            for (uint32_t i = 0; i < r; ++i) prod[i + 1] = P[i];
            reduce_phi(r, s, mask, prod, r);
            memcpy(P, prod, r * sizeof(uint32_t));
        }
    }
    free(prod);
}

/* u P(A) by Horner's rule: v = p_{r-1} u; v = v A + p_i u for i = r-2 .. 0,
 * where x A = f_1(x). */
void lfg_apply(uint32_t r, uint32_t s, uint32_t e, const uint32_t *W, const uint32_t *P, uint32_t *out)
{
    uint32_t mask = emask(e);
    uint32_t *v = (uint32_t *)malloc(r * sizeof(uint32_t));
    for (uint32_t k = 0; k < r; ++k) v[k] = (P[r - 1] * W[k]) & mask;
    for (int i = (int)r - 2; i >= 0; --i) {
        f1(r, s, mask, v);
        for (uint32_t k = 0; k < r; ++k) v[k] = (v[k] + P[i] * W[k]) & mask;
    }
    memcpy(out, v, r * sizeof(uint32_t));
    free(v);
}

/* c_J = (c - J d) mod m; only J mod m matters. */
uint32_t lfg_c_jump(uint32_t m, uint32_t d, uint32_t c, uint64_t jlo, uint64_t jhi)
{
    unsigned __int128 J = ((unsigned __int128)jhi << 64) | jlo;
    uint64_t jm = (uint64_t)(J % m);
    uint64_t sub = (jm * (uint64_t)d) % m;
    return (uint32_t)(((uint64_t)c + m - sub) % m);
}

/* f^J by the polynomial route: LFG part u P_J(A), c part in closed form. */
void lfg_jump(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d,
              const uint32_t *W, uint32_t c, uint64_t jlo, uint64_t jhi,
              uint32_t *W_out, uint32_t *c_out)
{
    uint32_t *P = (uint32_t *)malloc(r * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc(r * sizeof(uint32_t));
    lfg_xpow(r, s, e, jlo, jhi, P);
    lfg_apply(r, s, e, W, P, tmp);
    memcpy(W_out, tmp, r * sizeof(uint32_t));
    *c_out = lfg_c_jump(m, d, c, jlo, jhi);
    free(P);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Batch helpers: one call per test case.  State records are r + 1 words.   */
/* ------------------------------------------------------------------------ */
void lfg_jump_many(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d, uint64_t n,
                   const uint32_t *states_in, const uint64_t *jlo, const uint64_t *jhi,
                   uint32_t *states_out)
{
    for (uint64_t q = 0; q < n; ++q) {
        const uint32_t *si = states_in + (uint64_t)(r + 1) * q;
        uint32_t *so = states_out + (uint64_t)(r + 1) * q;
        lfg_jump(r, s, e, m, d, si, si[r], jlo[q], jhi[q], so, so + r);
    }
}

void lfg_draws_many(uint32_t r, uint32_t s, uint32_t e, uint32_t m, uint32_t d, uint64_t n,
                    const uint32_t *states_in, uint64_t count, uint32_t *out, uint64_t ld,
                    uint32_t *states_out)
{
    for (uint64_t q = 0; q < n; ++q) {
        const uint32_t *si = states_in + (uint64_t)(r + 1) * q;
        uint32_t *so = states_out ? states_out + (uint64_t)(r + 1) * q : 0;
        lfg_draws(r, s, e, m, d, si, si[r], count, out ? out + ld * q : 0, so, so ? so + r : 0);
    }
}

void lfg_xpow_many(uint32_t r, uint32_t s, uint32_t e, uint64_t n, const uint64_t *jlo,
                   const uint64_t *jhi, uint32_t *P)
{
    for (uint64_t q = 0; q < n; ++q) lfg_xpow(r, s, e, jlo[q], jhi[q], P + (uint64_t)r * q);
}
