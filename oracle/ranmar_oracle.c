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
 * Everything is written from the definitions, not from the printed listings:
 *   - the generator as a sequence (Sec. 2): x_n = x_{n-97} - x_{n-33} mod 1
 *     (mod 2^24 in integer form), c_n = c_{n-1} - d mod m, output x_n - c_n
 *     mod 1; the integer form takes c_n from its closed form (Sec. 3.2) and
 *     keeps the words in a ring indexed by the sequence number;
 *   - the initialisation (Appendix A) as its parts: the seed selects the
 *     starting values of two small generators, a lag-3 product generator
 *     modulo 179 and a linear congruential generator modulo 169; each step of
 *     the pair gives one bit, and 24 consecutive bits, first bit most
 *     significant, form one word of 24-bit precision;
 *   - the real-arithmetic form (the floating-point initialisation of Appendix
 *     A and the real-number generator) as a second, independent route: its own
 *     index arithmetic and generator stepping, words as sums of 2^-p, and the
 *     arithmetic sequence stepped in real numbers.  Sec. 3.1 (the isomorphism
 *     sigma) and Appendix A assert that the two routes agree exactly; the tests
 *     compare them, so a slip in either one shows;
 *   - the automaton state (u_1..u_97, c) and f applied literally (Sec. 2);
 *   - t^J mod phi(t) over Z/2^24 by binary powering, schoolbook products and
 *     generic long division by phi (Sec. 3.1, P_J; Sec. 4, Table 2);
 *   - u P_J(A) by Horner's rule (Sec. 3.1) and the closed-form c jump (Sec. 3.2).
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   - the canonical state is the automaton state (x_1, ..., x_97) with x_1 the
 *     oldest word, plus the integer numerator c' of c (0 <= c' < m);
 *   - the initialisation's words u_1..u_97 enter the sequence from the top
 *     down: the generator starts its two pointers at 97 and 33 and moves them
 *     down, so x_1 = u_97, ..., x_97 = u_1, and the first new word is
 *     u_97 - u_33;
 *   - the product generator's step is the product of the three previous
 *     values modulo 179 (both reductions are remainders; the printed Quotient
 *     would make seed 1 produce an all-zero state);
 *   - offset 0 is the state right after the initialisation; draw n (n >= 1)
 *     makes the new word and the new c first and outputs their difference.
 *
 * Parity status: every function below is pinned by the CPU tests except the
 * absolute values produced by the initialisation, which the paper prints no
 * example of ("parity unpinned" against any external source).  They are
 * pinned by the agreement of the two independent routes, by the index
 * arithmetic's bijection onto the generators' start values, by the product
 * generator's exponent form, by the congruential generator's closed form and
 * full period, and by the first draws read off the seeded words.
 */
#include <stdint.h>
#include <string.h>

/* Parameters of Sec. 2: lags (r, s) = (97, 33), precision e = 24,
 * (M, m, d) = (2^24, 2^24 - 3, 7654321/2^24), c = 362436/2^24. */
#define ORC_R 97
#define ORC_S 33
#define ORC_MASK 0xFFFFFFu
#define ORC_MOD 16777213u
#define ORC_D 7654321u
#define ORC_C0 362436u

/* Appendix A: seeds run up to 9 x 10^8.  Seed 0 would need the quotient of
 * the negative number s - 1, which the paper leaves undefined, so the range
 * used is [1, 9 x 10^8]. */
#define ORC_SEED_MAX 900000000

/* Appendix A: the initialisation draws 97 words of 24 bits each. */
#define ORC_SEED_BITS (97 * 24)

/* ======================================================================== */
/* Integer route.                                                           */
/* ======================================================================== */

/* Appendix A, start values.  Write q = s - 1 as q = 30082 a + b with
 * 0 <= b < 30082 = 178 * 169.  The high part a gives the product generator's
 * first two values i, j in [2, 178]; the low part b gives its third value k in
 * [1, 178] and the congruential generator's start l in [0, 168].
 * out = {i, j, k, l}; returns -1 for a seed outside [1, 9e8]. */
int orc_seed_setup(int64_t seed, int32_t out[4])
{
    if (seed < 1 || seed > ORC_SEED_MAX) return -1;
    int64_t q = seed - 1;
    int64_t a = q / 30082, b = q % 30082;
    out[0] = (int32_t)((a / 177) % 177 + 2);
    out[1] = (int32_t)(a % 177 + 2);
    out[2] = (int32_t)((b / 169) % 178 + 1);
    out[3] = (int32_t)(b % 169);
    return 0;
}

/* Appendix A, the two small generators, n = 1..count:
 *   m_n = m_{n-3} m_{n-2} m_{n-1} mod 179 with (m_{-2}, m_{-1}, m_0) = (i, j, k),
 *   l_n = 53 l_{n-1} + 1 mod 169          with l_0 = l.
 * Either output array may be NULL. */
void orc_seed_sequences(const int32_t start[4], int32_t count, int32_t *mseq, int32_t *lseq)
{
    int32_t m_prev[3] = {start[0], start[1], start[2]}; /* m_{n-3}, m_{n-2}, m_{n-1} */
    int32_t l_prev = start[3];
    for (int32_t n = 1; n <= count; ++n) {
        int32_t m_n = (int32_t)(((int64_t)m_prev[0] * m_prev[1] % 179) * m_prev[2] % 179);
        int32_t l_n = (53 * l_prev + 1) % 169;
        m_prev[0] = m_prev[1];
        m_prev[1] = m_prev[2];
        m_prev[2] = m_n;
        l_prev = l_n;
        if (mseq) mseq[n - 1] = m_n;
        if (lseq) lseq[n - 1] = l_n;
    }
}

/* Appendix A, the bit of step n: set when l_n m_n mod 64 lies in the upper
 * half [32, 64). */
static int seed_bit_of(int32_t m_n, int32_t l_n)
{
    return (l_n * m_n) % 64 >= 32;
}

/* Appendix A in integer form: word u_w (w = 1..97) is the 24-bit integer
 * whose binary digits, most significant first, are the bits of steps
 * 24(w-1)+1 .. 24w.  Fills u[1..97]; u[0] is unused and set to 0. */
int orc_seed_int(int64_t seed, uint32_t u[98])
{
    int32_t start[4];
    if (orc_seed_setup(seed, start)) return -1;
    int32_t mseq[ORC_SEED_BITS], lseq[ORC_SEED_BITS];
    orc_seed_sequences(start, ORC_SEED_BITS, mseq, lseq);
    u[0] = 0;
    for (int w = 1; w <= 97; ++w) {
        uint32_t word = 0;
        for (int p = 0; p < 24; ++p) {
            int n = 24 * (w - 1) + p; /* 0-based index of step 24(w-1)+p+1 */
            word = 2 * word + (uint32_t)seed_bit_of(mseq[n], lseq[n]);
        }
        u[w] = word;
    }
    return 0;
}

/* The canonical state after the initialisation (offset 0): the words enter
 * the sequence from the top down, x_1 = u_97, ..., x_97 = u_1, and c' = c_0. */
int orc_state_from_seed(int64_t seed, uint32_t W[97], uint32_t *c)
{
    uint32_t u[98];
    if (orc_seed_int(seed, u)) return -1;
    for (int k = 0; k < 97; ++k) W[k] = u[97 - k] & ORC_MASK;
    *c = ORC_C0;
    return 0;
}

/* Sec. 3.2: c'_n = (c'_0 - n d') mod m in closed form. */
static uint32_t c_after(uint32_t c0, uint64_t n)
{
    uint64_t sub = (n % ORC_MOD) * ORC_D % ORC_MOD;
    return (uint32_t)(((uint64_t)c0 + ORC_MOD - sub) % ORC_MOD);
}

/* Sec. 2 as a sequence: the state W holds x_1..x_97 (x_1 oldest).  Draw q
 * (q = 1..n) makes x_{97+q} = x_q - x_{q+64} mod 2^24 and outputs
 * y_q = x_{97+q} - c'_q mod 2^24.  The words live in a ring indexed by the
 * sequence number: x_t sits in slot (t - 1) mod 97, so the new word replaces
 * the one 97 places back.  The state after the draws (x_{n+1}..x_{n+97},
 * c'_n) is returned in Wout/cout (either may be NULL). */
void orc_state_draws(const uint32_t W[97], uint32_t c, uint64_t n, uint32_t *out,
                     uint32_t *Wout, uint32_t *cout)
{
    uint32_t ring[97];
    memcpy(ring, W, sizeof ring);
    for (uint64_t q = 1; q <= n; ++q) {
        uint64_t t = 97 + q;                           /* index of the new word */
        uint32_t x_old = ring[(t - 97 - 1) % 97];      /* x_{t-97} */
        uint32_t x_mid = ring[(t - 33 - 1) % 97];      /* x_{t-33} */
        uint32_t x_new = (x_old - x_mid) & ORC_MASK;
        ring[(t - 1) % 97] = x_new;
        if (out) out[q - 1] = (x_new - c_after(c, q)) & ORC_MASK;
    }
    if (Wout)
        for (int k = 0; k < 97; ++k) Wout[k] = ring[(n + (uint64_t)k) % 97];
    if (cout) *cout = c_after(c, n);
}

/* The integer generator from a seed: n draws after the initialisation. */
int orc_int_draws(int64_t seed, uint64_t n, uint32_t *out)
{
    uint32_t W[97], c;
    if (orc_state_from_seed(seed, W, &c)) return -1;
    orc_state_draws(W, c, n, out, 0, 0);
    return 0;
}

/* ======================================================================== */
/* Real route (double; every value is a multiple of 2^-24 in (-1, 2), so    */
/* the arithmetic is exact).  It repeats none of the integer route's code.  */
/* ======================================================================== */

/* The small generators of the real initialisation, kept as a running triple
 * of the product generator and the congruential value. */
typedef struct {
    long p0, p1, p2; /* the last three values of the product generator, oldest first */
    long lc;         /* the congruential generator's last value */
} real_init_gen;

/* One step of the pair; returns the bit the step contributes. */
static int real_init_next(real_init_gen *g)
{
    long prod = g->p0 * g->p1 * g->p2 % 179; /* < 179^3, no overflow */
    g->p0 = g->p1;
    g->p1 = g->p2;
    g->p2 = prod;
    g->lc = (g->lc * 53 + 1) % 169;
    return (int)((prod * g->lc) % 64 / 32); /* 1 exactly in the upper half */
}

/* Floating-point initialisation: word w (w = 1..97) is the binary fraction
 * 0.b_1 b_2 ... b_24 of the next 24 bits, summed as b_p 2^-p.  The start
 * values come from nested quotients: i and j from the quotient of s - 1 by
 * 30082 (its quotient and remainder by 177), k and l from the remainder (its
 * quotient by 169 taken mod 178, and its remainder by 169).  Fills u[1..97]. */
int orc_seed_real(int64_t seed, double u[98])
{
    if (seed < 1 || seed > ORC_SEED_MAX) return -1;
    long q = (long)(seed - 1);
    long hi = q / 30082, lo = q - 30082 * hi;
    real_init_gen g;
    g.p0 = 2 + (q / (30082L * 177)) % 177; /* quotient of hi by 177, mod 177 */
    g.p1 = 2 + hi % 177;
    g.p2 = 1 + (lo / 169) % 178;
    g.lc = lo % 169;
    u[0] = 0.0;
    for (int w = 1; w <= 97; ++w) {
        double frac = 0.0;
        for (int p = 1; p <= 24; ++p) {
            double weight = 1.0;
            for (int h = 0; h < p; ++h) weight *= 0.5;
            frac += real_init_next(&g) ? weight : 0.0;
        }
        u[w] = frac;
    }
    return 0;
}

/* The real-number generator (the form Algorithm 1 computes), as a sequence:
 * x_t = x_{t-97} - x_{t-33} mod 1, c_t = c_{t-1} - d mod m (m = 16777213/2^24,
 * d = 7654321/2^24, c_0 = 362436/2^24), output x_t - c_t mod 1.  The seeded
 * words enter from the top down (x_1 = u_97). */
int orc_real_draws(int64_t seed, uint64_t n, double *out)
{
    double u[98];
    if (orc_seed_real(seed, u)) return -1;
    const double two24 = 16777216.0;
    const double d = 7654321.0 / two24, mreal = 16777213.0 / two24;
    double c = 362436.0 / two24;
    double x[97];
    for (int k = 0; k < 97; ++k) x[k] = u[97 - k];
    /* x[] is a window that slides by one word per draw: x[0] = x_{t-97}. */
    for (uint64_t q = 0; q < n; ++q) {
        double nw = x[0] - x[64];
        if (nw < 0.0) nw += 1.0;
        for (int k = 0; k < 96; ++k) x[k] = x[k + 1];
        x[96] = nw;
        c -= d;
        if (c < 0.0) c += mreal;
        double y = nw - c;
        if (y < 0.0) y += 1.0;
        out[q] = y;
    }
    return 0;
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
