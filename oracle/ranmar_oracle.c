/*
 * RANMAR oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of what the
 * RANMAR hot path computes, written from Haramoto & Suzuki, "Making the RANMAR
 * pseudorandom number generator in LAMMPS up to four times faster, with an
 * implementation of jump-ahead" (arXiv 2512.00093).  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant generator with the GPU library; the two
 * are compared against each other, never built on each other.
 *
 * Contents, each following the passage it cites:
 *   - real-arithmetic seeding and draws      (Appendix A / Algorithm 3 in its
 *                                             real form; Algorithm 1)
 *   - integer seeding and draws, w = 32      (Algorithm 3; Algorithm 2)
 *   - the automaton state (u_1..u_97, c)     (Sec. 2, finite automaton; Sec. 3.1)
 *   - t^J mod phi(t) over Z/2^24 by binary
 *     powering, schoolbook products and
 *     generic long division by phi           (Sec. 3.1, P_J; Sec. 4, Table 2)
 *   - uP_J(A) by Horner's rule                (Sec. 3.1, Horner formula)
 *   - closed-form jump of c                   (Sec. 3.2)
 *   - literal J-fold stepping of f           (Sec. 2, f^J)
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   - the canonical state is the automaton state u = (u_1, ..., u_97) with
 *     u_1 the oldest word, plus the integer numerator c' of c (0 <= c' < m);
 *   - Algorithm 3's inner multiplicative step is read as
 *     Remainder(Remainder(i*j,179)*k,179): the printed Quotient would make
 *     seed 1 produce an all-zero state;
 *   - offset 0 is the state right after Algorithm 3; draw n (n >= 1) steps the
 *     state first and then outputs (x_new - c_new) mod 2^24, as Algorithms 1
 *     and 2 do.
 *
 * Parity status: every function below is pinned by the CPU tests except the
 * absolute values produced by the seeding procedure, which the paper prints
 * no example of ("parity unpinned" against any external source; they are
 * pinned only by real == integer agreement and the Remainder reading).
 */
#include <stdint.h>
#include <string.h>

/* Parameters of Sec. 2: lags (r, s) = (97, 33), precision e = 24,
 * (M, m, d) = (2^24, 2^24 - 3, 7654321/2^24), c = 362436/2^24. */
#define ORC_R 97
#define ORC_S 33
#define ORC_M24 16777216.0
#define ORC_MASK 0xFFFFFFu
#define ORC_MOD 16777213u
#define ORC_D 7654321u
#define ORC_C0 362436u

/* ------------------------------------------------------------------------ */
/* Appendix A: the index set-up shared by both forms of the initialisation.  */
/* ------------------------------------------------------------------------ */
static int seed_indices(int64_t seed, long *i, long *j, long *k, long *l)
{
    /* The paper allows 0 <= s <= 9e8 but never defines Quotient/Remainder of
     * the negative number s-1 = -1, so seed 0 is rejected. */
    if (seed < 1 || seed > 900000000) return -1;
    long ij = (long)((seed - 1) / 30082);
    long kl = (long)((seed - 1) - 30082 * ij);
    *i = (ij / 177) % 177 + 2;
    *j = ij % 177 + 2;
    *k = (kl / 169) % 178 + 1;
    *l = kl % 169;
    return 0;
}

/* One step of the initialisation's two small generators; returns the bit. */
static int seed_bit(long *i, long *j, long *k, long *l)
{
    long m = ((*i * *j) % 179) * *k % 179; /* Remainder reading */
    *i = *j;
    *j = *k;
    *k = m;
    *l = (53 * *l + 1) % 169;
    return (*l * m) % 64 >= 32;
}

/* Real-number initialisation (the form Algorithm 3 re-implements; its
 * comments give the real form: t starts at 0.5 and is halved each step).
 * Fills u[1..97]. */
int orc_seed_real(int64_t seed, double u[98])
{
    long i, j, k, l;
    if (seed_indices(seed, &i, &j, &k, &l)) return -1;
    u[0] = 0.0;
    for (int ii = 1; ii <= 97; ++ii) {
        double s = 0.0, t = 0.5;
        for (int jj = 1; jj <= 24; ++jj) {
            if (seed_bit(&i, &j, &k, &l)) s = s + t;
            t = 0.5 * t;
        }
        u[ii] = s;
    }
    return 0;
}

/* Algorithm 3 with w = 32: t = 2^31 halved each step, u = s / 2^(w-24). */
int orc_seed_int(int64_t seed, uint32_t u[98])
{
    long i, j, k, l;
    if (seed_indices(seed, &i, &j, &k, &l)) return -1;
    u[0] = 0;
    for (int ii = 1; ii <= 97; ++ii) {
        uint32_t s = 0, t = 0x80000000u;
        for (int jj = 1; jj <= 24; ++jj) {
            if (seed_bit(&i, &j, &k, &l)) s = s + t;
            t = t / 2;
        }
        u[ii] = s >> 8;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: RANMAR in real arithmetic (double; every value is a multiple */
/* of 2^-24 in (-1, 2), so the arithmetic is exact).                         */
/* ------------------------------------------------------------------------ */
int orc_real_draws(int64_t seed, uint64_t n, double *out)
{
    double u[98];
    if (orc_seed_real(seed, u)) return -1;
    double c = 362436.0 / ORC_M24, cd = 7654321.0 / ORC_M24, cm = 16777213.0 / ORC_M24;
    int i = 97, j = 33;
    for (uint64_t q = 0; q < n; ++q) {
        double y = u[i] - u[j];
        if (y < 0) y = y + 1.0;
        u[i] = y;
        i = i - 1;
        if (i == 0) i = 97;
        j = j - 1;
        if (j == 0) j = 97;
        c = c - cd;
        if (c < 0) c = c + cm;
        y = y - c;
        if (y < 0) y = y + 1.0;
        out[q] = y;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: RANMAR in modular arithmetic with 32-bit unsigned words.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t u[98]; /* u[1..97] */
    uint32_t v;     /* numerator of c, 0 <= v < m */
    int i, j;
} alg2_state;

static uint32_t alg2_draw(alg2_state *st)
{
    uint32_t x = st->u[st->i] - st->u[st->j];
    st->u[st->i] = x;
    st->i = st->i - 1;
    if (st->i == 0) st->i = 97;
    st->j = st->j - 1;
    if (st->j == 0) st->j = 97;
    st->v = st->v + (ORC_MOD - ORC_D);
    if (st->v >= ORC_MOD) st->v = st->v - ORC_MOD;
    return (x - st->v) & ORC_MASK;
}

int orc_int_draws(int64_t seed, uint64_t n, uint32_t *out)
{
    alg2_state st;
    if (orc_seed_int(seed, st.u)) return -1;
    st.v = ORC_C0;
    st.i = 97;
    st.j = 33;
    for (uint64_t q = 0; q < n; ++q) out[q] = alg2_draw(&st);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The automaton state of Sec. 2 / Sec. 3.1: W[0..96] = (u_1, ..., u_97),    */
/* u_1 oldest, plus c'.  Algorithm 2 keeps the same words in a circular      */
/* array whose oldest entry is at index i and whose lag-33 entry is at j.    */
/* ------------------------------------------------------------------------ */
static int wrap97(int idx)
{
    while (idx < 1) idx += 97;
    while (idx > 97) idx -= 97;
    return idx;
}

static void alg2_to_state(const alg2_state *st, uint32_t W[97], uint32_t *c)
{
    for (int k = 0; k < 97; ++k) W[k] = st->u[wrap97(st->i - k)] & ORC_MASK;
    *c = st->v;
}

static void state_to_alg2(const uint32_t W[97], uint32_t c, alg2_state *st)
{
    st->i = 97;
    st->j = 33;
    st->u[0] = 0;
    for (int k = 0; k < 97; ++k) st->u[97 - k] = W[k];
    st->v = c;
}

/* State right after Algorithm 3 (offset 0). */
int orc_state_from_seed(int64_t seed, uint32_t W[97], uint32_t *c)
{
    alg2_state st;
    if (orc_seed_int(seed, st.u)) return -1;
    st.v = ORC_C0;
    st.i = 97;
    st.j = 33;
    alg2_to_state(&st, W, c);
    return 0;
}

/* n draws of Algorithm 2 started from a canonical state; the state after the
 * n draws is returned in Wout/cout (either may be NULL). */
void orc_state_draws(const uint32_t W[97], uint32_t c, uint64_t n, uint32_t *out,
                     uint32_t *Wout, uint32_t *cout)
{
    alg2_state st;
    state_to_alg2(W, c, &st);
    for (uint64_t q = 0; q < n; ++q) {
        uint32_t y = alg2_draw(&st);
        if (out) out[q] = y;
    }
    uint32_t Wt[97], ct;
    alg2_to_state(&st, Wt, &ct);
    if (Wout) memcpy(Wout, Wt, sizeof Wt);
    if (cout) *cout = ct;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2: the transition f = (f_1, f_2) applied literally J times.          */
/* f_1(u_1..u_97) = (u_2, ..., u_97, u_1 - u_65);  f_2(c) = c - d mod m.     */
/* ------------------------------------------------------------------------ */
static void F1(uint32_t u[97])
{
    uint32_t nw = (u[0] - u[ORC_R - ORC_S]) & ORC_MASK; /* u_1 - u_{r-s+1} */
    memmove(u, u + 1, 96 * sizeof(uint32_t));
    u[96] = nw;
}

void orc_step(const uint32_t W[97], uint32_t c, uint64_t J, uint32_t Wout[97], uint32_t *cout)
{
    uint32_t u[97];
    memcpy(u, W, sizeof u);
    for (uint64_t q = 0; q < J; ++q) {
        F1(u);
        c = (c >= ORC_D) ? c - ORC_D : c + ORC_MOD - ORC_D;
    }
    memcpy(Wout, u, sizeof u);
    *cout = c;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: P_J(t) = t^J mod phi(t) in (Z/2^24)[t], phi = t^97 + t^64 - 1.  */
/* Polynomials are coefficient arrays, index = power of t.                   */
/* ------------------------------------------------------------------------ */

/* phi as a list of (exponent, coefficient) terms; monic of degree 97. */
static const int PHI_EXP[3] = {0, 64, 97};
static const int PHI_COEF[3] = {-1, 1, 1};

/* Schoolbook product followed by long division by the monic phi. */
void orc_poly_mulmod(const uint32_t a[97], const uint32_t b[97], uint32_t out[97])
{
    uint32_t prod[193];
    memset(prod, 0, sizeof prod);
    for (int i = 0; i < 97; ++i)
        for (int j = 0; j < 97; ++j)
            prod[i + j] = (prod[i + j] + (a[i] & ORC_MASK) * (b[j] & ORC_MASK)) & ORC_MASK;
    for (int k = 192; k >= 97; --k) {
        uint32_t q = prod[k]; /* leading coefficient; phi is monic */
        for (int e = 0; e < 3; ++e) {
            int pos = k - 97 + PHI_EXP[e];
            prod[pos] = (prod[pos] - q * (uint32_t)PHI_COEF[e]) & ORC_MASK;
        }
    }
    for (int i = 0; i < 97; ++i) out[i] = prod[i];
}

/* Left-to-right binary powering of t, J = jhi * 2^64 + jlo. */
void orc_xpow(uint64_t jlo, uint64_t jhi, uint32_t P[97])
{
    uint32_t tpoly[97];
    memset(P, 0, 97 * sizeof(uint32_t));
    memset(tpoly, 0, sizeof tpoly);
    P[0] = 1;
    tpoly[1] = 1;
    for (int bit = 127; bit >= 0; --bit) {
        uint32_t tmp[97];
        orc_poly_mulmod(P, P, tmp);
        memcpy(P, tmp, sizeof tmp);
        int set = bit >= 64 ? (int)((jhi >> (bit - 64)) & 1) : (int)((jlo >> bit) & 1);
        if (set) {
            orc_poly_mulmod(P, tpoly, tmp);
            memcpy(P, tmp, sizeof tmp);
        }
    }
}

/* Horner's rule for u P(A) (Sec. 3.1), with xA = F1(x). */
void orc_apply(const uint32_t W[97], const uint32_t P[97], uint32_t out[97])
{
    uint32_t v[97];
    for (int k = 0; k < 97; ++k) v[k] = (P[96] * W[k]) & ORC_MASK;
    for (int i = 95; i >= 0; --i) {
        F1(v);
        for (int k = 0; k < 97; ++k) v[k] = (v[k] + P[i] * W[k]) & ORC_MASK;
    }
    memcpy(out, v, sizeof v);
}

/* Sec. 3.2: c'_J = (c'_0 - J d') mod m; only J mod m is needed. */
uint32_t orc_c_jump(uint32_t c, uint64_t jlo, uint64_t jhi)
{
    unsigned __int128 J = ((unsigned __int128)jhi << 64) | jlo;
    uint64_t jm = (uint64_t)(J % ORC_MOD);
    uint64_t sub = (jm * ORC_D) % ORC_MOD;
    return (uint32_t)(((uint64_t)c + ORC_MOD - sub) % ORC_MOD);
}

/* f^J of the automaton: LFG part by P_J(A), c part in closed form. */
void orc_jump(const uint32_t W[97], uint32_t c, uint64_t jlo, uint64_t jhi,
              uint32_t Wout[97], uint32_t *cout)
{
    uint32_t P[97], tmp[97];
    orc_xpow(jlo, jhi, P);
    orc_apply(W, P, tmp);
    memcpy(Wout, tmp, sizeof tmp);
    *cout = orc_c_jump(c, jlo, jhi);
}

/* ------------------------------------------------------------------------ */
/* Batch helpers so that the Python test harness makes one call per case.   */
/* A state record is 98 words: W[0..96] then c.                              */
/* ------------------------------------------------------------------------ */
int orc_seed_jump_many(uint64_t n, const int64_t *seeds, const uint64_t *jlo,
                       const uint64_t *jhi, uint32_t *states)
{
    for (uint64_t r = 0; r < n; ++r) {
        uint32_t W[97], c;
        if (orc_state_from_seed(seeds[r], W, &c)) return -1;
        orc_jump(W, c, jlo ? jlo[r] : 0, jhi ? jhi[r] : 0, states + 98 * r, states + 98 * r + 97);
    }
    return 0;
}

void orc_draws_many(uint64_t n, const uint32_t *states_in, uint64_t count,
                    uint32_t *out, uint64_t ld, uint32_t *states_out)
{
    for (uint64_t r = 0; r < n; ++r) {
        const uint32_t *s = states_in + 98 * r;
        orc_state_draws(s, s[97], count, out ? out + ld * r : 0,
                        states_out ? states_out + 98 * r : 0,
                        states_out ? states_out + 98 * r + 97 : 0);
    }
}

void orc_xpow_many(uint64_t n, const uint64_t *jlo, const uint64_t *jhi, uint32_t *P)
{
    for (uint64_t r = 0; r < n; ++r) orc_xpow(jlo[r], jhi[r], P + 97 * r);
}
