/*
 * pcpd_oracle.c -- plain CPU oracle for the multispin Monte Carlo sweep of the
 * 1+1-dimensional n-tuple contact process with diffusion (DP n=1, PCPD n=2,
 * TCPD n=3, QCPD n=4), from R.D. Schram, "Reaction-diffusion model Monte
 * Carlo simulations on the GPU" (arXiv:1301.6082). The paper develops the
 * PCPD and names DP, TCPD and QCPD as direct extensions (Sec. 1).
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no code, header, table or constant generator with the
 * HIP path; both are written independently from the same definition.
 *
 * What it computes, and where each piece comes from:
 *
 *   Reactions and rates ............ paper Sec. 2, eq. (1):
 *        AA0 -> AAA and 0AA -> AAA each with rate (1-p)(1-d)/2,
 *        AA -> 00 with rate p(1-d), A0 <-> 0A with rate d.
 *   Per-attempt semantics ........... paper Algorithm 1 (sequential PCPD): one
 *        attempt at site j first diffuses (swap j, j+1) with probability d;
 *        otherwise, if j and j+1 hold a pair, the pair annihilates with
 *        probability p, else a particle is created at j-1 or at j+2 with
 *        equal probability. Generalised to an n-tuple j..j+n-1: diffusion
 *        still swaps (j, j+1), annihilation clears the tuple, fission fills
 *        j-1 ("low") or j+n ("high"). Fission onto an occupied site changes
 *        nothing.
 *   Site selection .................. paper Sec. 3: the ring is cut into equal
 *        parts of B sites and every part is updated at the same randomly
 *        chosen local site. One substep draws an offset o uniform in [0,B)
 *        and applies the rule at j = k*B + o for every block k. Windows
 *        j-1..j+n of different blocks are disjoint when B >= n+2, so their
 *        order within a substep does not matter. B substeps make one Monte
 *        Carlo step (L attempts per sample, time +1). With B = L this is
 *        exactly Algorithm 1.
 *   Multispin samples ............... paper Sec. 4 (classical multispin): 64
 *        independent lattices per plane, one per bit of a 64-bit word. Here
 *        each sample is stored as its own byte array and updated with
 *        branches, one sample at a time.
 *   Random numbers .................. Philox-4x32-10 (Salmon, Moraes, Dror,
 *        Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) replaces
 *        the paper's Tausworthe generator (Sec. 3). Key (seed, stream_id).
 *        Counter (c0, c1, c2, c3) with s = substep index = t*B + b:
 *          offset of (plane q, substep s):  (0, 8q+7, lo32 s, hi32 s),
 *                                           o = (x0 * B) >> 32
 *          window k, draw 0:  (k, 8q+0, lo32 s, hi32 s) -> X1_D, X2_D
 *          window k, draw 1:  (k, 8q+1, ...)            -> X1_A, X2_A
 *          window k, draw 2:  (k, 8q+2, ...)            -> R, gD, gA
 *          with m = 4 decorrelation bits also
 *          window k, draw 3:  (k, 8q+3, ...)            -> X3_D, X4_D
 *          window k, draw 4:  (k, 8q+4, ...)            -> X3_A, X4_A
 *        with X1 = x0 | x1<<32, X2 = x2 | x3<<32 (X3, X4 likewise), R = x0 |
 *        x1<<32, gD = x2, gA = x3. Bit b of each 64-bit word belongs to sample b.
 *   Probability-q decisions ......... the paper builds probability-d and
 *        probability-p bits from AND/OR of random words (Sec. 4.2) and from
 *        one word-wide comparison RNG() < 4p shared by all bits (Sec. 4.3).
 *        Generalised here to any q in [0,1]: sample b draws the (32+m)-bit
 *        integer U_b = u_b * 2^32 + g, where u_b is the m-bit number whose
 *        bits, most significant first, are bit b of X1 .. Xm (m independent
 *        bits per sample: the paper's decorrelation bits, m = 2 by default,
 *        or 4) and g is shared by the 64 samples of that word, and decides
 *        U_b < K with K = rint(q * 2^(32+m)). R_b = 1 means fission high.
 *   Observables ..................... paper Sec. 5.3: particle density and
 *        pair density. Per sample, N = number of occupied sites and
 *        N_pair = number of nearest-neighbour pairs (j, j+1 mod L) that are
 *        both occupied.
 *
 * Readings where the paper is silent or inconsistent (listed with reasons in
 * the design notes): periodic boundary, fully occupied start, Algorithm 2's
 * annihilation must clear (not keep) the pair, Algorithm 2's fission-low must
 * OR into site i-1, the "1" of RNG() < 4p is an all-ones word.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Philox-4x32-10, as published by Salmon et al. (SC'11): ten rounds of
 *   (L0', R0', L1', R1') with
 *   hi0:lo0 = M0 * c0, hi1:lo1 = M1 * c2,
 *   c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
 * the key incremented by the Weyl constants between rounds.
 * ------------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; round++) {
        uint64_t prod0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* K = rint(q * 2^34), the integer threshold of a probability-q decision.
 * Returns UINT64_MAX for q outside [0,1] or not finite. */
uint64_t orc_threshold(double q)
{
    if (!(q >= 0.0 && q <= 1.0))
        return UINT64_MAX;
    return (uint64_t)rint(ldexp(q, 34));
}

/* Decision bit of sample b: U_b < K with U_b = (2*bit_b(x1) + bit_b(x2))*2^32 + g. */
int orc_decide(uint64_t x1, uint64_t x2, uint32_t g, uint64_t K, int b)
{
    uint64_t u = 2u * ((x1 >> b) & 1u) + ((x2 >> b) & 1u);
    uint64_t U = (u << 32) + (uint64_t)g;
    return U < K ? 1 : 0;
}

/* K = rint(q * 2^(32+m)) for m decorrelation bits (2 or 4); UINT64_MAX for a
 * bad q or m. */
uint64_t orc_threshold_m(double q, int m)
{
    if (!(q >= 0.0 && q <= 1.0) || (m != 2 && m != 4))
        return UINT64_MAX;
    return (uint64_t)rint(ldexp(q, 32 + m));
}

/* Decision bit of sample b with m bits: U_b = u * 2^32 + g, u = bit b of
 * x[0] .. x[m-1] read as an m-bit number, x[0] most significant. */
int orc_decide_m(const uint64_t *x, int m, uint32_t g, uint64_t K, int b)
{
    uint64_t u = 0;
    int i;
    for (i = 0; i < m; i++)
        u = 2u * u + ((x[i] >> b) & 1u);
    return ((u << 32) + (uint64_t)g) < K ? 1 : 0;
}

/* Offset o of substep s of plane q: uniform in [0, B). */
uint32_t orc_offset(uint32_t seed, uint32_t stream, uint32_t plane, uint64_t s, uint32_t B)
{
    uint32_t ctr[4] = {0u, (plane << 3) | 7u, (uint32_t)s, (uint32_t)(s >> 32)};
    uint32_t key[2] = {seed, stream};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return (uint32_t)(((uint64_t)x[0] * (uint64_t)B) >> 32);
}

/* The three draws of window k of plane q in substep s. */
typedef struct {
    uint64_t xd[4], xa[4], r;  /* X1..Xm of the diffusion and annihilation decisions */
    uint32_t gd, ga;
} orc_draws;

static orc_draws window_draws(uint32_t seed, uint32_t stream, uint32_t plane, uint64_t s,
                              uint32_t k, int m)
{
    orc_draws w;
    uint32_t key[2] = {seed, stream};
    uint32_t ctr[4], x[4];
    ctr[0] = k;
    ctr[2] = (uint32_t)s;
    ctr[3] = (uint32_t)(s >> 32);

    ctr[1] = (plane << 3) | 0u;
    orc_philox4x32_10(ctr, key, x);
    w.xd[0] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    w.xd[1] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);

    ctr[1] = (plane << 3) | 1u;
    orc_philox4x32_10(ctr, key, x);
    w.xa[0] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    w.xa[1] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);

    ctr[1] = (plane << 3) | 2u;
    orc_philox4x32_10(ctr, key, x);
    w.r = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    w.gd = x[2];
    w.ga = x[3];

    w.xd[2] = w.xd[3] = w.xa[2] = w.xa[3] = 0;
    if (m == 4) {
        ctr[1] = (plane << 3) | 3u;
        orc_philox4x32_10(ctr, key, x);
        w.xd[2] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        w.xd[3] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
        ctr[1] = (plane << 3) | 4u;
        orc_philox4x32_10(ctr, key, x);
        w.xa[2] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        w.xa[3] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
    }
    return w;
}

/* One attempt on one sample at window site j (Algorithm 1, n-tuple form).
 * q is the sample's lattice, one byte per site, 0 = empty, 1 = particle. */
static void attempt(int n, uint8_t *q, uint64_t L, uint64_t j, int D, int A, int R)
{
    uint64_t here = j % L;
    uint64_t right = (j + 1) % L;
    int i;
    if (D) { /* diffusion A0 <-> 0A: swap sites j and j+1 */
        uint8_t tmp = q[here];
        q[here] = q[right];
        q[right] = tmp;
        return;
    }
    for (i = 0; i < n; i++) /* is j..j+n-1 an n-tuple of particles? */
        if (!q[(j + (uint64_t)i) % L])
            return;
    if (A) { /* annihilation: the tuple disappears */
        for (i = 0; i < n; i++)
            q[(j + (uint64_t)i) % L] = 0;
        return;
    }
    if (R) /* fission high: a particle appears right of the tuple */
        q[(j + (uint64_t)n) % L] = 1;
    else /* fission low: a particle appears left of the tuple */
        q[(j + L - 1) % L] = 1;
}

/* Apply the rule to a lone window state, for table checks: bit i of `window`
 * is site j-1+i (i = 0..n+1). Returns the new window. The window is treated
 * as an open segment (no wrap). */
uint32_t orc_rule_window(int n, uint32_t window, int D, int A, int R)
{
    uint8_t q[8];
    int i;
    uint32_t outw = 0;
    if (n < 1 || n > 5)
        return 0xffffffffu;
    for (i = 0; i < n + 2; i++)
        q[i] = (uint8_t)((window >> i) & 1u);
    /* a ring of n+2 sites with j = 1 touches each site exactly once */
    attempt(n, q, (uint64_t)(n + 2), 1, D, A, R);
    for (i = 0; i < n + 2; i++)
        outw |= (uint32_t)q[i] << i;
    return outw;
}

typedef struct {
    int32_t n;          /* tuple size: 1 DP, 2 PCPD, 3 TCPD, 4 QCPD */
    uint32_t B;         /* block width */
    uint64_t L;         /* ring length */
    uint32_t seed;      /* Philox key word 0 */
    uint32_t stream;    /* Philox key word 1 */
    uint32_t plane;     /* plane index q */
    double p, d;        /* rates of eq. (1) */
    uint64_t samples;   /* which of the 64 samples to simulate (bit b = sample b) */
    int32_t init;       /* 0 full, 1 empty, 2 from init_words */
    const uint64_t *init_words; /* L words, natural site order, if init == 2 */
    uint64_t t0;        /* Monte Carlo step at which the lattice is given */
    uint32_t n_times;   /* record times, strictly increasing, >= t0 */
    const uint64_t *times;
    uint64_t *words_out;   /* L words: final lattice (bits of unsimulated samples are 0) */
    uint64_t *n_out;       /* [n_times][64] particles per sample */
    uint64_t *pair_out;    /* [n_times][64] pairs per sample */
    int32_t connected;     /* 1: the 64 bits form one joined lattice (orc_simulate_connected) */
    int32_t mask_bits;     /* decorrelation bits m of every decision: 2 (also for 0) or 4 */
} orc_params;

static int orc_simulate_connected(const orc_params *P);

/* Error codes: 0 ok, -1 invalid arguments, -2 out of memory. */
int orc_simulate(const orc_params *P)
{
    uint8_t *lat[64];
    int nsim = 0, idx[64];
    int b, rc = 0;
    uint64_t Kd, Kp, t, j;
    uint32_t r, k;
    uint64_t nblocks;
    int m;

    if (!P || P->n < 1 || P->n > 4 || P->B < (uint32_t)(P->n + 2) || P->L < P->B ||
        P->L % P->B != 0 || (P->L / P->B) > 0xffffffffull || P->plane >= (1u << 29))
        return -1;
    m = P->mask_bits ? P->mask_bits : 2;
    Kd = orc_threshold_m(P->d, m);
    Kp = orc_threshold_m(P->p, m);
    if (Kd == UINT64_MAX || Kp == UINT64_MAX)
        return -1;
    if (P->init == 2 && !P->init_words)
        return -1;
    for (r = 0; r < P->n_times; r++)
        if (P->times[r] < P->t0 || (r > 0 && P->times[r] <= P->times[r - 1]))
            return -1;

    if (P->connected)
        return orc_simulate_connected(P);
    nblocks = P->L / P->B;
    for (b = 0; b < 64; b++) {
        lat[b] = NULL;
        if ((P->samples >> b) & 1u)
            idx[nsim++] = b;
    }
    for (b = 0; b < nsim; b++) {
        lat[idx[b]] = (uint8_t *)malloc(P->L);
        if (!lat[idx[b]]) {
            rc = -2;
            goto done;
        }
        for (j = 0; j < P->L; j++) {
            if (P->init == 0)
                lat[idx[b]][j] = 1;
            else if (P->init == 1)
                lat[idx[b]][j] = 0;
            else
                lat[idx[b]][j] = (uint8_t)((P->init_words[j] >> idx[b]) & 1u);
        }
    }

    t = P->t0;
    for (r = 0; r < P->n_times; r++) {
        /* advance to the record time, one Monte Carlo step (B substeps) at a time */
        for (; t < P->times[r]; t++) {
            uint32_t sub;
            for (sub = 0; sub < P->B; sub++) {
                uint64_t s = t * (uint64_t)P->B + sub;
                uint32_t o = orc_offset(P->seed, P->stream, P->plane, s, P->B);
                for (k = 0; k < nblocks; k++) {
                    orc_draws w = window_draws(P->seed, P->stream, P->plane, s, k, m);
                    uint64_t site = (uint64_t)k * P->B + o;
                    for (b = 0; b < nsim; b++) {
                        int sb = idx[b];
                        int D = orc_decide_m(w.xd, m, w.gd, Kd, sb);
                        int A = orc_decide_m(w.xa, m, w.ga, Kp, sb);
                        int R = (int)((w.r >> sb) & 1u);
                        attempt(P->n, lat[sb], P->L, site, D, A, R);
                    }
                }
            }
        }
        /* record */
        for (b = 0; b < 64; b++) {
            if (P->n_out)
                P->n_out[(uint64_t)r * 64 + b] = 0;
            if (P->pair_out)
                P->pair_out[(uint64_t)r * 64 + b] = 0;
        }
        for (b = 0; b < nsim; b++) {
            int sb = idx[b];
            uint64_t cnt = 0, pairs = 0;
            for (j = 0; j < P->L; j++) {
                cnt += lat[sb][j];
                pairs += (uint64_t)(lat[sb][j] & lat[sb][(j + 1) % P->L]);
            }
            if (P->n_out)
                P->n_out[(uint64_t)r * 64 + sb] = cnt;
            if (P->pair_out)
                P->pair_out[(uint64_t)r * 64 + sb] = pairs;
        }
    }

    if (P->words_out) {
        for (j = 0; j < P->L; j++) {
            uint64_t w = 0;
            for (b = 0; b < nsim; b++)
                w |= (uint64_t)lat[idx[b]][j] << idx[b];
            P->words_out[j] = w;
        }
    }
done:
    for (b = 0; b < 64; b++)
        free(lat[b]);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Connected multispin lattice (paper Sec. 4, second paragraph, and the layout
 * of its Figs. 2-3): instead of 64 independent rings, the 64 bits of a plane
 * are joined into ONE ring of M = 64 L sites. Site g = b*L + j is bit b of
 * word j, so the sites held by one word are L apart (the paper's L/N_r for a
 * lattice of M sites and N_r = 64 bits). Neighbours follow the global site
 * order: after word L-1 of bit b comes word 0 of bit b+1, and after bit 63
 * comes bit 0 (the ring closes). A window that runs past the last word of the
 * plane therefore continues in the next bit of the first words -- the bit
 * rotation at the seam that connects the lattices.
 *
 * Site selection is the Sec. 3 scheme on the joined ring: M is cut into M/B
 * blocks, global block K = b*(L/B) + k (k = the word block, b = the bit), and
 * substep s attempts every block at its local site o (the same draw as in the
 * classical layout), i.e. at global site g = K*B + o = b*L + k*B + o. The
 * decision bits of that window are bit b of the masks of word window k
 * (the same Philox counters as the classical layout): each global window
 * reads its own bit, as each sample does in the classical layout.
 * Observables per bit column b (sites b*L .. b*L+L-1): particles, and pairs
 * (g, g+1) with g in the column (the pair leaving the column's last site
 * pairs it with the first site of column b+1).
 * ------------------------------------------------------------------------- */

/* One substep s of the Sec. 3 scheme on a joined ring of M = 64 L sites held
 * as bytes (q[g] for global site g), with m decorrelation bits. */
static void connected_substep_m(int n, uint32_t B, uint64_t L, uint32_t seed, uint32_t stream,
                                uint32_t plane, uint64_t Kd, uint64_t Kp, uint64_t s, uint8_t *q,
                                int m)
{
    uint64_t nblocks = L / B, M = 64u * L, k;
    uint32_t o = orc_offset(seed, stream, plane, s, B);
    int b;
    for (k = 0; k < nblocks; k++) {
        orc_draws w = window_draws(seed, stream, plane, s, (uint32_t)k, m);
        for (b = 0; b < 64; b++) {
            uint64_t g = (uint64_t)b * L + k * B + o; /* global block b*nblocks + k */
            int D = orc_decide_m(w.xd, m, w.gd, Kd, b);
            int A = orc_decide_m(w.xa, m, w.ga, Kp, b);
            int R = (int)((w.r >> b) & 1u);
            attempt(n, q, M, g, D, A, R);
        }
    }
}

/* The same with m = 2 (exported for the tests of the layout). */
void orc_connected_substep(int n, uint32_t B, uint64_t L, uint32_t seed, uint32_t stream,
                           uint32_t plane, uint64_t Kd, uint64_t Kp, uint64_t s, uint8_t *q)
{
    connected_substep_m(n, B, L, seed, stream, plane, Kd, Kp, s, q, 2);
}

static int orc_simulate_connected(const orc_params *P)
{
    uint64_t M = 64u * P->L, Kd, Kp, t, j, g;
    uint8_t *q;
    uint32_t r, sub;
    int b, m = P->mask_bits ? P->mask_bits : 2;
    Kd = orc_threshold_m(P->d, m);
    Kp = orc_threshold_m(P->p, m);
    if (Kd == UINT64_MAX || Kp == UINT64_MAX)
        return -1;
    q = (uint8_t *)malloc(M);
    if (!q)
        return -2;
    for (b = 0; b < 64; b++)
        for (j = 0; j < P->L; j++) {
            g = (uint64_t)b * P->L + j;
            if (P->init == 0)
                q[g] = 1;
            else if (P->init == 1)
                q[g] = 0;
            else
                q[g] = (uint8_t)((P->init_words[j] >> b) & 1u);
        }
    t = P->t0;
    for (r = 0; r < P->n_times; r++) {
        for (; t < P->times[r]; t++)
            for (sub = 0; sub < P->B; sub++)
                connected_substep_m(P->n, P->B, P->L, P->seed, P->stream, P->plane, Kd, Kp,
                                    t * (uint64_t)P->B + sub, q, m);
        for (b = 0; b < 64; b++) {
            uint64_t cnt = 0, pairs = 0;
            for (j = 0; j < P->L; j++) {
                g = (uint64_t)b * P->L + j;
                cnt += q[g];
                pairs += (uint64_t)(q[g] & q[(g + 1) % M]);
            }
            if (P->n_out)
                P->n_out[(uint64_t)r * 64 + b] = cnt;
            if (P->pair_out)
                P->pair_out[(uint64_t)r * 64 + b] = pairs;
        }
    }
    if (P->words_out)
        for (j = 0; j < P->L; j++) {
            uint64_t w = 0;
            for (b = 0; b < 64; b++)
                w |= (uint64_t)q[(uint64_t)b * P->L + j] << b;
            P->words_out[j] = w;
        }
    free(q);
    return 0;
}

/* Independent (instance, plane) units in parallel, one per thread; there is
 * no threading inside a unit. n_threads <= 0 uses the OpenMP default.
 * Returns the first nonzero unit status, or 0. */
int orc_simulate_many(const orc_params *P, int32_t count, int32_t n_threads, int32_t *status)
{
    int32_t i;
    int rc = 0;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < count; i++)
        status[i] = orc_simulate(&P[i]);
    (void)n_threads;
    for (i = 0; i < count; i++)
        if (status[i] != 0 && rc == 0)
            rc = status[i];
    return rc;
}

/* Threads the OpenMP runtime would use for orc_simulate_many. */
int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
