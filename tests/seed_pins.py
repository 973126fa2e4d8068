"""Checks of the initialisation (Appendix A, Algorithm 3) that rest on
arithmetic facts rather than on the oracle's own formulas.

The paper prints no seeded state, so the absolute words stay unpinned against
any outside source.  What the printed constants do fix is checked here:
- 30082 = 178 * 169, so the low part of s - 1 maps one-to-one onto the start
  values (k, l) in [1, 178] x [0, 168];
- the high part is below 177^2, so (i, j) is its two base-177 digits (plus 2)
  and the whole map seed -> (i, j, k, l) is one-to-one;
- 179 is prime and the product generator starts on non-zero residues, so with
  a primitive root g its values are g^(e_n) where the exponents follow the
  three-term additive recurrence e_n = e_(n-1) + e_(n-2) + e_(n-3) mod 178;
- the congruential generator l -> 53 l + 1 mod 169 has the closed form
  l_n = 53^n l_0 + (53^n - 1)/52 and, by the Hull-Dobell theorem (53 - 1 is a
  multiple of 13, the only prime factor of 169; the increment 1 is a unit),
  full period 169;
- the generator's first draws read the seeded words from the top down: draw q
  (q <= 33) is u_(98-q) - u_(34-q) - c_q mod 2^24.

Each check takes callables for the routine it tests and returns the list of
failed check names (empty when all hold), so the pin tests run it on the
oracle and the mutation tests on copies with planted mistakes.
"""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MASK = (1 << 24) - 1


def golden():
    out = {}
    with open(os.path.join(GOLDEN, "paper_parameters.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split(None, 1)
                out[k] = v.strip()
    return out


def check_setup_low_part(setup):
    """Within one block of 30082 consecutive seeds, (i, j) is fixed and (k, l)
    runs once over [1, 178] x [0, 168]."""
    g = golden()
    split, kmod, lmod = int(g["seed_split"]), int(g["k_mod"]), int(g["l_mod"])
    fails = []
    if split != kmod * lmod:
        fails.append("split_is_k_times_l")
    want = {(k, l) for k in range(1, kmod + 1) for l in range(lmod)}
    for a in (0, 12345, 29917):
        seen, ij = [], set()
        for b in range(split):
            i, j, k, l = setup(a * split + b + 1)
            seen.append((k, l))
            ij.add((i, j))
        if len(ij) != 1 or set(seen) != want or len(seen) != len(set(seen)):
            fails.append("low_part_bijection")
            break
    return fails


def check_setup_high_part(setup):
    """The high part a = (s - 1) // 30082 takes every value up to
    (9e8 - 1) // 30082 < 177^2; (i, j) must then differ for every a and lie in
    the non-zero residues mod 179, and the product generator's three start
    values are never all 1 (which would make it constant)."""
    g = golden()
    split, radix, pmod = int(g["seed_split"]), int(g["ij_radix"]), int(g["prod_mod"])
    top = (int(g["seed_max"]) - 1) // split
    fails = []
    if top >= radix * radix:
        fails.append("high_part_fits_two_digits")
    seen = set()
    for a in range(top + 1):
        i, j, k, l = setup(a * split + 1)
        if not (1 <= i < pmod and 1 <= j < pmod and 1 <= k < pmod) or (i, j, k) == (1, 1, 1):
            fails.append("start_values_in_unit_group")
            break
        seen.add((i, j))
    if len(seen) != top + 1:
        fails.append("high_part_injective")
    # The last seed (a partial block) stays in range too.
    i, j, k, l = setup(int(g["seed_max"]))
    if not (1 <= i < pmod and 1 <= j < pmod and 1 <= k < pmod and 0 <= l < int(g["l_mod"])):
        fails.append("last_seed_in_range")
    return fails


def _primitive_root_logs(p):
    """A primitive root of the prime p and its discrete-log table."""
    for gen in range(2, p):
        logs, v = {}, 1
        for e in range(p - 1):
            logs.setdefault(v, e)
            v = v * gen % p
        if len(logs) == p - 1:
            return gen, logs
    raise AssertionError("no primitive root")


def check_product_generator(setup, sequences, seeds, steps=None):
    """The product generator in exponent form: with g primitive mod 179,
    m_n = g^(e_n) and e_n = e_(n-1) + e_(n-2) + e_(n-3) mod 178, started from
    the logarithms of (i, j, k)."""
    g = golden()
    p = int(g["prod_mod"])
    steps = steps or 97 * int(g["bits_per_word"])
    gen, logs = _primitive_root_logs(p)
    for s in seeds:
        start = setup(s)
        m, _ = sequences(start, steps)
        e = [logs[start[0] % p], logs[start[1] % p], logs[start[2] % p]] if all(
            v % p for v in start[:3]) else None
        if e is None:
            return ["product_generator_exponent_form"]
        for n in range(steps):
            e.append((e[-1] + e[-2] + e[-3]) % (p - 1))
            if int(m[n]) != pow(gen, e[-1], p):
                return ["product_generator_exponent_form"]
    return []


def check_congruential_generator(sequences):
    """Closed form l_n = 53^n l_0 + (53^n - 1)/(53 - 1) (mod 169) for every
    start, and full period 169."""
    g = golden()
    a, c, mod = int(g["lcg_mult"]), int(g["lcg_inc"]), int(g["l_mod"])
    fails = []
    for l0 in range(mod):
        _, l = sequences((2, 2, 1, l0), 2 * mod)
        for n in range(1, 2 * mod + 1):
            want = (pow(a, n) * l0 + c * ((pow(a, n) - 1) // (a - 1))) % mod
            if int(l[n - 1]) != want:
                fails.append("congruential_closed_form")
                return fails
        if sorted(int(v) for v in l[:mod]) != list(range(mod)) or int(l[mod - 1]) != l0:
            fails.append("congruential_full_period")
            return fails
    return fails


def check_first_draws(seed_int, int_draws, seeds):
    """The first 33 draws take their two words straight from the seeded array,
    from the top down: y_q = u_(98-q) - u_(34-q) - c_q mod 2^24 (the generator
    starts its pointers at 97 and 33; c_q = c_0 - q d mod m in closed form)."""
    g = golden()
    m, d, c0 = int(g["m"]), int(g["d_num"]), int(g["c_num"])
    for s in seeds:
        u = [int(v) for v in seed_int(s)]
        y = [int(v) for v in int_draws(s, 33)]
        for q in range(1, 34):
            want = (u[98 - q] - u[34 - q] - (c0 - q * d) % m) & MASK
            if y[q - 1] != want:
                return ["first_draws_from_seeded_words"]
    return []
