/*
 * ising_oracle.c -- plain CPU oracle for checkerboard Metropolis sweeps of
 * the 2D periodic square-lattice Ising model.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load this file's library. The product
 * path (the HIP library under paper_cs_0312006_amd/) shares no code with it.
 *
 * What is computed follows Tomov, McGuigan, Bennett, Smith, Spiletic,
 * "Benchmarking and Implementation of Probability-Based Simulations on
 * Programmable Graphics Cards" (2003):
 *   - energy and magnetisation of a state: Section 2.2, with Eq. (1) of
 *     Section 2.1 giving the expectation being estimated;
 *   - random initial state with spin-up probability p: Section 2.2;
 *   - checkerboard colouring, consecutive black/white passes: Section 2.2;
 *   - the four-step Metropolis decision with the Boltzmann ratio: Section 2.2.
 * Where the paper leaves a choice open the reading used here is written next
 * to the code (coupling J and field h, periodic boundaries, the random number
 * generator and its keying, R in (0,1], the lattice hash).
 *
 * Everything is deliberately plain: one Philox call per site (the group of
 * four sites that share a call recomputes it), canonical int8 +-1 storage in
 * row-major order, no blocking. OpenMP splits rows within one colour, which
 * is legal because same-coloured sites never neighbour each other.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-4)

/* Largest side accepted: the Philox counter's first word holds site/8 and
 * must fit 32 bits, and the sweep index t must fit 32 bits as well. */
#define ORACLE_MAX_L 65536u

static int g_threads = 1;

int oracle_set_threads(int n)
{
    if (n < 1) return ORACLE_EINVAL;
    g_threads = n;
    return ORACLE_OK;
}

int oracle_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------
 * Random numbers. The paper draws R from a linear congruential generator
 * (Section 2.1) whose constants it does not give, so the stream cannot be
 * reproduced. Here the draw is Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011): a keyed bijection
 * on four 32-bit words, ten rounds, each round multiplying words 0 and 2 by
 * fixed constants and mixing the high halves with words 1, 3 and the key;
 * the key is advanced by two Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The 32-bit uniform used at site (i, j) of an L x L lattice, sweep t,
 * colour c, domain d (0 = Metropolis decision, 1 = initial state).
 * Sites of one colour are numbered ord = (i*L + j) / 2, which for even L is
 * a bijection from that colour onto [0, L*L/2). Four consecutive ords share
 * one Philox call with counter (ord/4, t, c, d) and key (seed low, seed high);
 * the site takes output word ord % 4. */
uint32_t oracle_draw(uint64_t seed, uint32_t L, uint32_t t, uint32_t c, uint32_t d,
                     uint32_t i, uint32_t j)
{
    uint64_t ord = ((uint64_t)i * (uint64_t)L + (uint64_t)j) >> 1;
    uint32_t ctr[4] = {(uint32_t)(ord >> 2), t, c, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[ord & 3u];
}

/* ------------------------------------------------------------------------
 * Metropolis acceptance (Section 2.2, steps 2-4). With coupling J and field
 * h the energy is E = -J sum_<jk> s_j s_k - h sum_j s_j (the paper's energy
 * is the case J = 1, h = 0); flipping spin s whose four neighbours sum to n
 * changes it by dE = 2 s (J n + h). The move is accepted outright when
 * dE < 0; otherwise a uniform R is drawn and the move accepted when
 * R <= exp(-dE / T) (Boltzmann constant 1, T in units of J).
 *
 * Reading of R in [0, 1]: R = (u + 1) / 2^32 with u the 32-bit draw, so
 * R <= p  <=>  u < floor(p * 2^32). The threshold for each (s, n) is stored
 * as that integer, in [0, 2^32]; dE <= 0 gives 2^32 (for dE = 0 the ratio is
 * exactly 1, so the move is always taken either way).
 *
 * Table index: [si * 5 + ni] with si = 0 for s = -1, 1 for s = +1 and
 * ni = (n + 4) / 2 for n in {-4, -2, 0, 2, 4}.
 * ---------------------------------------------------------------------- */
int oracle_threshold_table(double J, double h, double T, uint64_t thr[10])
{
    if (!(isfinite(J) && isfinite(h) && isfinite(T) && T > 0.0)) return ORACLE_EINVAL;
    for (int si = 0; si < 2; ++si) {
        double s = si ? 1.0 : -1.0;
        for (int ni = 0; ni < 5; ++ni) {
            double n = (double)(2 * ni - 4);
            double dE = 2.0 * s * (J * n + h);
            uint64_t v;
            if (dE <= 0.0)
                v = (uint64_t)1 << 32;
            else
                v = (uint64_t)floor(exp(-dE / T) * 4294967296.0);
            thr[si * 5 + ni] = v;
        }
    }
    return ORACLE_OK;
}

static int valid_side(uint32_t L) { return L >= 2 && (L % 2) == 0 && L <= ORACLE_MAX_L; }

/* Random initial state (Section 2.2): each spin points up with probability
 * p_up, decided by the domain-1 draw of sweep 0 at the site's own colour:
 * up iff u < floor(p_up * 2^32). Output: canonical row-major int8, +1 / -1. */
int oracle_init(uint32_t L, uint64_t seed, double p_up, int8_t *s)
{
    if (!valid_side(L) || !(p_up >= 0.0 && p_up <= 1.0) || !s) return ORACLE_EINVAL;
    uint64_t pthr = (uint64_t)floor(p_up * 4294967296.0);
    int rows = (int)L;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int i = 0; i < rows; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            uint32_t c = ((uint32_t)i + j) & 1u;
            uint32_t u = oracle_draw(seed, L, 0, c, 1, (uint32_t)i, j);
            s[(size_t)i * L + j] = ((uint64_t)u < pthr) ? (int8_t)1 : (int8_t)-1;
        }
    }
    return ORACLE_OK;
}

/* One pass over all sites of colour c = (i + j) mod 2 at sweep t, in place
 * (Section 2.2: the checkerboard makes the order within a colour irrelevant,
 * since a site's four neighbours all have the other colour). Periodic
 * boundaries. */
int oracle_half_sweep(uint32_t L, const uint64_t thr[10], uint64_t seed, uint32_t t,
                      uint32_t c, int8_t *s)
{
    if (!valid_side(L) || c > 1 || !s || !thr) return ORACLE_EINVAL;
    int rows = (int)L;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int ii = 0; ii < rows; ++ii) {
        uint32_t i = (uint32_t)ii;
        uint32_t up = (i + L - 1) % L, dn = (i + 1) % L;
        for (uint32_t j = 0; j < L; ++j) {
            if (((i + j) & 1u) != c) continue;
            uint32_t lf = (j + L - 1) % L, rt = (j + 1) % L;
            int n = s[(size_t)up * L + j] + s[(size_t)dn * L + j] + s[(size_t)i * L + lf] +
                    s[(size_t)i * L + rt];
            int8_t me = s[(size_t)i * L + j];
            int si = me > 0 ? 1 : 0;
            int ni = (n + 4) / 2;
            uint32_t u = oracle_draw(seed, L, t, c, 0, i, j);
            if ((uint64_t)u < thr[si * 5 + ni]) s[(size_t)i * L + j] = (int8_t)(-me);
        }
    }
    return ORACLE_OK;
}

/* Integer observables of a state (Section 2.2): the bond sum
 * B = sum_{i,j} s(i,j) (s(i,j+1) + s(i+1,j)), periodic, which counts each
 * lattice edge once (so the paper's energy is -B, and in general
 * E = -J B - h M), and the magnetisation M = (#up) - (#down) = sum s. */
void oracle_observables(uint32_t L, const int8_t *s, int64_t *B, int64_t *M)
{
    int64_t b = 0, m = 0;
    int rows = (int)L;
#pragma omp parallel for schedule(static) reduction(+ : b, m) num_threads(g_threads)
    for (int ii = 0; ii < rows; ++ii) {
        uint32_t i = (uint32_t)ii;
        uint32_t dn = (i + 1) % L;
        for (uint32_t j = 0; j < L; ++j) {
            int me = s[(size_t)i * L + j];
            int right = s[(size_t)i * L + (j + 1) % L];
            int down = s[(size_t)dn * L + j];
            b += (int64_t)(me * (right + down));
            m += me;
        }
    }
    *B = b;
    *M = m;
}

/* n full sweeps t = t0 .. t0+n-1; a sweep is the colour-0 ("black",
 * i + j even) pass followed by the colour-1 pass. After each sweep the bond
 * sum and magnetisation are stored in B[k], M[k] (either may be NULL). */
int oracle_run(uint32_t L, double J, double h, double T, uint64_t seed, uint64_t t0,
               uint64_t n, int8_t *s, int64_t *B, int64_t *M)
{
    uint64_t thr[10];
    if (!valid_side(L) || !s) return ORACLE_EINVAL;
    if (oracle_threshold_table(J, h, T, thr) != ORACLE_OK) return ORACLE_EINVAL;
    if (t0 + n > ((uint64_t)1 << 32)) return ORACLE_ERANGE;
    for (uint64_t k = 0; k < n; ++k) {
        uint32_t t = (uint32_t)(t0 + k);
        oracle_half_sweep(L, thr, seed, t, 0, s);
        oracle_half_sweep(L, thr, seed, t, 1, s);
        if (B || M) {
            int64_t b, m;
            oracle_observables(L, s, &b, &m);
            if (B) B[k] = b;
            if (M) M[k] = m;
        }
    }
    return ORACLE_OK;
}

/* FNV-1a, 64-bit, over a byte string (offset basis 0xcbf29ce484222325,
 * prime 0x100000001b3). Applied to the canonical lattice bytes, where +1 is
 * 0x01 and -1 is 0xFF, row by row. */
uint64_t oracle_fnv1a64(const uint8_t *p, size_t n)
{
    uint64_t hsh = 0xcbf29ce484222325ull;
    for (size_t k = 0; k < n; ++k) {
        hsh ^= (uint64_t)p[k];
        hsh *= 0x100000001b3ull;
    }
    return hsh;
}

/* Light-cone restriction, for checking single sites of lattices too large
 * to simulate whole. A W x W window whose top-left corner is global site
 * (i0, j0) is evolved with exactly the rule above, using global coordinates
 * for colours and draws. A window site can be updated only if it and its
 * four neighbours lie in the window and are still exact; otherwise it is
 * marked inexact. valid[] (W*W bytes) returns 1 for sites whose value is
 * exact after the n sweeps. win[] holds the window's canonical int8 spins on
 * entry (the true state at sweep t0) and on return. */
int oracle_window_run(uint32_t L, double J, double h, double T, uint64_t seed, uint64_t t0,
                      uint64_t n, uint32_t i0, uint32_t j0, uint32_t W, int8_t *win,
                      uint8_t *valid)
{
    uint64_t thr[10];
    if (!valid_side(L) || W < 1 || W > L || i0 >= L || j0 >= L || !win || !valid)
        return ORACLE_EINVAL;
    if (oracle_threshold_table(J, h, T, thr) != ORACLE_OK) return ORACLE_EINVAL;
    if (t0 + n > ((uint64_t)1 << 32)) return ORACLE_ERANGE;
    memset(valid, 1, (size_t)W * W);
    int rows = (int)W;
    for (uint64_t k = 0; k < n; ++k) {
        uint32_t t = (uint32_t)(t0 + k);
        for (uint32_t c = 0; c < 2; ++c) {
#pragma omp parallel for schedule(static) num_threads(g_threads)
            for (int aa = 0; aa < rows; ++aa) {
                uint32_t a = (uint32_t)aa;
                uint32_t gi = (i0 + a) % L;
                for (uint32_t b = 0; b < W; ++b) {
                    uint32_t gj = (j0 + b) % L;
                    if (((gi + gj) & 1u) != c) continue;
                    size_t at = (size_t)a * W + b;
                    if (!valid[at]) continue;
                    if (a == 0 || b == 0 || a + 1 == W || b + 1 == W ||
                        !valid[at - W] || !valid[at + W] || !valid[at - 1] || !valid[at + 1]) {
                        valid[at] = 0;
                        continue;
                    }
                    int nsum = win[at - W] + win[at + W] + win[at - 1] + win[at + 1];
                    int8_t me = win[at];
                    int si = me > 0 ? 1 : 0;
                    int ni = (nsum + 4) / 2;
                    uint32_t u = oracle_draw(seed, L, t, c, 0, gi, gj);
                    if ((uint64_t)u < thr[si * 5 + ni]) win[at] = (int8_t)(-me);
                }
            }
        }
    }
    return ORACLE_OK;
}

/* Initial state of a window only (same rule as oracle_init). */
int oracle_init_window(uint32_t L, uint64_t seed, double p_up, uint32_t i0, uint32_t j0,
                       uint32_t W, int8_t *win)
{
    if (!valid_side(L) || W < 1 || W > L || i0 >= L || j0 >= L || !win ||
        !(p_up >= 0.0 && p_up <= 1.0))
        return ORACLE_EINVAL;
    uint64_t pthr = (uint64_t)floor(p_up * 4294967296.0);
    for (uint32_t a = 0; a < W; ++a) {
        uint32_t gi = (i0 + a) % L;
        for (uint32_t b = 0; b < W; ++b) {
            uint32_t gj = (j0 + b) % L;
            uint32_t u = oracle_draw(seed, L, 0, (gi + gj) & 1u, 1, gi, gj);
            win[(size_t)a * W + b] = ((uint64_t)u < pthr) ? (int8_t)1 : (int8_t)-1;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Creutz's deterministic checkerboard dynamics (Section 2.2 names it as the
 * faster alternative that needs no high-quality random numbers). Reading
 * used here: every site carries a demon energy d in units of 4J (h = 0,
 * J > 0), 0 <= d <= 255. A pass over colour c flips each of its sites iff
 * its demon can pay for the move, e = dE / 4J = s * n / 2 (n the neighbour
 * sum, so e in {-2, -1, 0, 1, 2}): flip iff e <= d and d - e <= 255, and
 * then d -= e. A sweep is the colour-0 pass followed by the colour-1 pass.
 * Spin energy plus 4J times the demon total is conserved exactly, and each
 * pass is its own inverse.
 * Demons use the canonical row-major layout of the spins (one byte a site).
 * ---------------------------------------------------------------------- */
int oracle_creutz_half_sweep(uint32_t L, uint32_t c, int8_t *s, uint8_t *d)
{
    if (!valid_side(L) || c > 1 || !s || !d) return ORACLE_EINVAL;
    int rows = (int)L;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int ii = 0; ii < rows; ++ii) {
        uint32_t i = (uint32_t)ii;
        uint32_t up = (i + L - 1) % L, dn = (i + 1) % L;
        for (uint32_t j = 0; j < L; ++j) {
            if (((i + j) & 1u) != c) continue;
            uint32_t lf = (j + L - 1) % L, rt = (j + 1) % L;
            int n = s[(size_t)up * L + j] + s[(size_t)dn * L + j] + s[(size_t)i * L + lf] +
                    s[(size_t)i * L + rt];
            size_t at = (size_t)i * L + j;
            int e = s[at] * n / 2;
            int dem = d[at];
            if (e <= dem && dem - e <= 255) {
                s[at] = (int8_t)(-s[at]);
                d[at] = (uint8_t)(dem - e);
            }
        }
    }
    return ORACLE_OK;
}

/* Sum of the demon energies (units of 4J). */
int64_t oracle_demon_sum(uint32_t L, const uint8_t *d)
{
    int64_t t = 0;
    for (size_t k = 0; k < (size_t)L * L; ++k) t += d[k];
    return t;
}

/* n Creutz sweeps; after each, B, M and the demon total are stored in B[k],
 * M[k], D[k] (any may be NULL). reverse != 0 runs the inverse sweeps
 * (colour 1 then colour 0), which undo forward sweeps exactly. */
int oracle_creutz_run(uint32_t L, uint64_t n, int reverse, int8_t *s, uint8_t *d, int64_t *B, int64_t *M,
                      int64_t *D)
{
    if (!valid_side(L) || !s || !d) return ORACLE_EINVAL;
    for (uint64_t k = 0; k < n; ++k) {
        oracle_creutz_half_sweep(L, reverse ? 1u : 0u, s, d);
        oracle_creutz_half_sweep(L, reverse ? 0u : 1u, s, d);
        if (B || M) {
            int64_t b, m;
            oracle_observables(L, s, &b, &m);
            if (B) B[k] = b;
            if (M) M[k] = m;
        }
        if (D) D[k] = oracle_demon_sum(L, d);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Site percolation in a porous medium (Section 2.3).
 *
 * Medium: an L x L lattice with open (non-periodic) boundaries. Each site
 * draws R and is a pore iff R <= P (the porosity). As for the Ising draws,
 * R = (u + 1) / 2^32 with u a 32-bit Philox4x32-10 output, so the site is a
 * pore iff u < floor(P * 2^32). Reading used here for the keying: site
 * ord = i*L + j takes word ord % 4 of counter (ord / 4, 0, 0, 2) under key
 * (seed low, seed high); domain 2 keeps these draws apart from the Ising
 * ones (domains 0 and 1).
 *
 * Invasion: the cluster starts at the invasion point(s), pores only, and
 * spreads in passes; pass k adds every pore that shares an edge with a
 * site already in the cluster. Reading used here: the invasion source is
 * either every pore of row 0 (the medium's top face, so the cluster spans
 * when it reaches row L-1) or one point (i0, j0). The arrival pass of a
 * site is its breadth-first distance from the sources through pores, -1 if
 * it is never invaded; the steady state is reached after (max arrival)
 * passes, and one more pass changes nothing.
 * ---------------------------------------------------------------------- */
#define ORACLE_PERC_TOP_ROW 0u
#define ORACLE_PERC_POINT 1u

int oracle_perc_medium(uint32_t L, double P, uint64_t seed, uint8_t *pore)
{
    if (L < 1 || L > ORACLE_MAX_L || !(P >= 0.0 && P <= 1.0) || !pore) return ORACLE_EINVAL;
    uint64_t pthr = (uint64_t)floor(P * 4294967296.0);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int rows = (int)L;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int i = 0; i < rows; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            uint64_t ord = (uint64_t)i * L + j;
            uint32_t ctr[4] = {(uint32_t)(ord >> 2), 0u, 0u, 2u};
            uint32_t out[4];
            oracle_philox4x32_10(ctr, key, out);
            pore[ord] = ((uint64_t)out[ord & 3u] < pthr) ? 1u : 0u;
        }
    }
    return ORACLE_OK;
}

/* Arrival passes by breadth-first search from the sources (a FIFO queue of
 * site indices; each site enters it once). */
int oracle_perc_invade(uint32_t L, const uint8_t *pore, uint32_t source, uint32_t i0, uint32_t j0,
                       int32_t *arrival, uint32_t *queue)
{
    if (L < 1 || L > ORACLE_MAX_L || !pore || !arrival || !queue) return ORACLE_EINVAL;
    if (source > ORACLE_PERC_POINT || (source == ORACLE_PERC_POINT && (i0 >= L || j0 >= L)))
        return ORACLE_EINVAL;
    size_t N = (size_t)L * L, head = 0, tail = 0;
    for (size_t k = 0; k < N; ++k) arrival[k] = -1;
    if (source == ORACLE_PERC_TOP_ROW) {
        for (uint32_t j = 0; j < L; ++j)
            if (pore[j]) {
                arrival[j] = 0;
                queue[tail++] = j;
            }
    } else {
        size_t at = (size_t)i0 * L + j0;
        if (pore[at]) {
            arrival[at] = 0;
            queue[tail++] = (uint32_t)at;
        }
    }
    while (head < tail) {
        size_t at = queue[head++];
        uint32_t i = (uint32_t)(at / L), j = (uint32_t)(at % L);
        size_t nb[4];
        int cnt = 0;
        if (i > 0) nb[cnt++] = at - L;
        if (i + 1 < L) nb[cnt++] = at + L;
        if (j > 0) nb[cnt++] = at - 1;
        if (j + 1 < L) nb[cnt++] = at + 1;
        for (int k = 0; k < cnt; ++k) {
            if (pore[nb[k]] && arrival[nb[k]] < 0) {
                arrival[nb[k]] = arrival[at] + 1;
                queue[tail++] = (uint32_t)nb[k];
            }
        }
    }
    return ORACLE_OK;
}

/* Summary of an arrival map: invaded sites, steady-state pass count (max
 * arrival, 0 for an empty cluster), and spanning bits: 1 = the cluster
 * holds a site of row 0 and one of row L-1, 2 = of column 0 and column L-1. */
void oracle_perc_summary(uint32_t L, const int32_t *arrival, uint64_t *invaded, int32_t *max_arrival,
                         uint32_t *spans)
{
    uint64_t n = 0;
    int32_t mx = 0;
    int top = 0, bottom = 0, left = 0, right = 0;
    for (uint32_t i = 0; i < L; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            int32_t a = arrival[(size_t)i * L + j];
            if (a < 0) continue;
            ++n;
            if (a > mx) mx = a;
            top |= i == 0;
            bottom |= i == L - 1;
            left |= j == 0;
            right |= j == L - 1;
        }
    }
    *invaded = n;
    *max_arrival = mx;
    *spans = (uint32_t)((top && bottom) ? 1 : 0) | (uint32_t)((left && right) ? 2 : 0);
}
