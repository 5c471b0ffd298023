/*
 * muca_oracle.c -- plain, slow, single-threaded CPU oracle for parallel
 * multicanonical (MUCA) and multimagnetic (MUMA) simulations
 * (Zierenberg, Marenz, Janke, "Scaling Properties of Parallelized
 * Multicanonical Simulations", arXiv:1312.2213).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call
 * this file; only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
 * bench.py use it.  It shares no code, header, table or constant generator
 * with the HIP library: every step below is written out from the paper and
 * from the published definitions it relies on.
 *
 * Floating point is IEEE double throughout; build with -ffp-contract=off so
 * that no fused multiply-add changes a rounding.
 *
 * What each function follows:
 *   orc_philox        Philox4x32-10, Salmon et al., SC'11 ("Parallel random
 *                     numbers: as easy as 1, 2, 3"), Sec. 3.2 / Table 2.
 *   orc_init_lattice  p independent realisations with the same weights
 *                     (paper, parallel-scheme paragraph and Fig. 1).
 *   orc_sweeps        Metropolis with the MUCA weight W(E) (Eq. 1) or the
 *                     MUMA weight exp(-beta E) W(M) (Eq. 3); 2D Ising
 *                     H = -J sum s_i s_j and q-state Potts
 *                     H = -J sum delta(s_i,s_j) (model paragraphs).
 *   orc_recursion     weight recursion using the accumulated statistics of
 *                     all earlier iterations in log weights (paper, paragraph
 *                     after Eq. 2); it reduces to W/H on the first step.
 *   orc_flatness      "flat energy distribution" stopping rule (paper,
 *                     parallel-scheme paragraph).
 *   orc_reweight      reweighting to canonical expectation values (Eq. 2).
 *   orc_sweeps_em,    multimagnetic runs (Eq. 3) with the joint histogram of
 *   orc_reweight_em   E and the flattened M, reweighted to the canonical
 *                     ensemble at another inverse temperature (Eq. 2 with the
 *                     MUMA weight in place of W(E)).
 *   orc_polymer_*     bead-spring homopolymer with LJ + FENE (Eq. 7) and
 *                     single-monomer shift moves; optionally the paper's full
 *                     move set (shift, spherical rotation, double bridging,
 *                     polymer paragraph), in the forms stated at the moves.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10.  Round: (hi0,lo0)=M0*x0, (hi1,lo1)=M1*x2;                 */
/* x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0); key bumped by the Weyl constants    */
/* between rounds.  Constants from the Random123 paper.                      */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = (uint32_t)(seed & 0xffffffffu);
    uint32_t k1 = (uint32_t)(seed >> 32);
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0, p1;
        uint32_t hi0, lo0, hi1, lo1;
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        hi0 = (uint32_t)(p0 >> 32);
        lo0 = (uint32_t)p0;
        hi1 = (uint32_t)(p1 >> 32);
        lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Stream layout: counter = (chain, sweep, block, tag), key = seed. */
#define ORC_TAG_SWEEP 0u
#define ORC_TAG_INIT 1u
#define ORC_TAG_ROT 2u    /* polymer spherical rotations */
#define ORC_TAG_BRIDGE 3u /* polymer double bridging */

static void draw(uint64_t seed, uint32_t chain, uint32_t sweep, uint32_t block,
                 uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4];
    ctr[0] = chain;
    ctr[1] = sweep;
    ctr[2] = block;
    ctr[3] = tag;
    orc_philox(ctr, seed, out);
}

/* ------------------------------------------------------------------------ */
/* Lattice models                                                            */
/* ------------------------------------------------------------------------ */
enum { ORC_ISING = 0, ORC_POTTS = 1, ORC_MUMA = 2 };

typedef struct {
    int32_t model;    /* ORC_ISING, ORC_POTTS, ORC_MUMA                  */
    int32_t L;        /* linear size, periodic L x L                     */
    int32_t q;        /* Potts states                                    */
    int32_t n_chains; /* p independent realisations                      */
    uint64_t seed;
    int32_t lo, hi;   /* binned range: Ising E, Potts E_unsat, MUMA M    */
    double beta;      /* MUMA: fixed inverse temperature                 */
} orc_lattice;

/* bin width of the binned quantity, in its own units */
static int32_t bin_step(int32_t model)
{
    if (model == ORC_ISING)
        return 4; /* E = -sum s_i s_j changes in steps of 4 */
    if (model == ORC_POTTS)
        return 1; /* E_unsat: one bin per integer */
    return 2;     /* M changes in steps of 2 */
}

int32_t orc_nbins(const orc_lattice *c)
{
    return (c->hi - c->lo) / bin_step(c->model) + 1;
}

/* threshold-table columns per bin */
int32_t orc_ncols(int32_t model)
{
    if (model == ORC_ISING)
        return 5; /* n_aligned = 0..4            */
    if (model == ORC_POTTS)
        return 9; /* dE_unsat = -4..4           */
    return 10;    /* (n_aligned, spin sign)     */
}

/* Values of the binned quantity that no configuration takes (Omega = 0);
 * checked by enumeration in the tests.  1 = reachable. */
void orc_reachable(const orc_lattice *c, uint8_t *mask)
{
    int32_t N = c->L * c->L;
    int32_t B = orc_nbins(c);
    int32_t b;
    for (b = 0; b < B; ++b) {
        int32_t v = c->lo + b * bin_step(c->model);
        int ok = 1;
        if (c->model == ORC_ISING) {
            if (v == -2 * N + 4 || v == 2 * N - 4)
                ok = 0;
        } else if (c->model == ORC_POTTS) {
            if (c->q == 2) {
                if ((v & 1) || v == 2 || v == 2 * N - 2)
                    ok = 0;
            } else {
                if (v == 1 || v == 2 || v == 3 || v == 5)
                    ok = 0;
            }
        }
        mask[b] = (uint8_t)ok;
    }
}

static int32_t site(int32_t L, int32_t y, int32_t x)
{
    y = (y + L) % L;
    x = (x + L) % L;
    return y * L + x;
}

/* Energy (Ising: -sum s_i s_j; Potts: number of unsatisfied bonds) and
 * magnetisation of one chain, each bond counted once (right, down). */
static void measure(const orc_lattice *c, const int8_t *s, int32_t *E, int32_t *M)
{
    int32_t L = c->L, y, x, e = 0, m = 0;
    for (y = 0; y < L; ++y)
        for (x = 0; x < L; ++x) {
            int32_t i = site(L, y, x);
            int32_t r = site(L, y, x + 1), d = site(L, y + 1, x);
            if (c->model == ORC_POTTS) {
                e += (s[i] != s[r]) + (s[i] != s[d]);
            } else {
                e -= s[i] * s[r] + s[i] * s[d];
                m += s[i];
            }
        }
    *E = e;
    *M = m;
}

void orc_measure(const orc_lattice *c, const int8_t *s, int32_t *E, int32_t *M)
{
    measure(c, s, E, M);
}

/* spins[chain][site]: Ising/MUMA +-1, Potts colour 0..q-1 (as unsigned bytes) */
void orc_init_lattice(const orc_lattice *c, int8_t *spins, int32_t *E, int32_t *M)
{
    int32_t N = c->L * c->L, ch, i;
    for (ch = 0; ch < c->n_chains; ++ch) {
        int8_t *s = spins + (int64_t)ch * N;
        uint32_t w[4];
        for (i = 0; i < N; ++i) {
            uint32_t r;
            if ((i & 3) == 0)
                draw(c->seed, (uint32_t)ch, 0u, (uint32_t)(i >> 2), ORC_TAG_INIT, w);
            r = w[i & 3];
            if (c->model == ORC_POTTS)
                s[i] = (int8_t)(((uint64_t)r * (uint64_t)c->q) >> 32);
            else
                s[i] = (r >> 31) ? (int8_t)1 : (int8_t)-1;
        }
        measure(c, s, &E[ch], &M[ch]);
    }
}

/* Acceptance threshold for a log-weight change D: the move is accepted iff
 * T == 0xffffffff or r < T, r a uniform 32-bit word, i.e. with probability
 * min(1, exp(D)) up to 2^-32. */
static uint32_t threshold(double D)
{
    double v;
    if (D >= 0.0)
        return 0xffffffffu;
    v = ldexp(exp(D), 32);
    if (v >= 4294967295.0)
        return 0xffffffffu;
    return (uint32_t)floor(v);
}

uint32_t orc_threshold(double D)
{
    return threshold(D);
}

/* T[b*ncols + j]: acceptance threshold from bin b for column j.
 *   Ising: j = n_aligned, dE = 4j - 8, target bin b + (j - 2).
 *   Potts: j = dE + 4 (dE = change of E_unsat), target bin b + dE.
 *   MUMA:  j = 2 n_aligned + (s_i == +1); dE = 4 n_aligned - 8; the flip
 *          changes M by -2 s_i, target bin b - s_i; the log weight change is
 *          lnW(M') - lnW(M) - beta dE (Eq. 3).
 * A target outside [lo, hi] gets T = 0 (never accepted). */
void orc_thresholds(const orc_lattice *c, const double *lnW, uint32_t *T)
{
    int32_t B = orc_nbins(c), nc = orc_ncols(c->model), b, j;
    for (b = 0; b < B; ++b)
        for (j = 0; j < nc; ++j) {
            int32_t t;
            double D;
            if (c->model == ORC_ISING) {
                t = b + (j - 2);
                if (t < 0 || t >= B) {
                    T[b * nc + j] = 0u;
                    continue;
                }
                D = lnW[t] - lnW[b];
            } else if (c->model == ORC_POTTS) {
                t = b + (j - 4);
                if (t < 0 || t >= B) {
                    T[b * nc + j] = 0u;
                    continue;
                }
                D = lnW[t] - lnW[b];
            } else {
                int32_t n = j / 2, up = j % 2;
                int32_t dE = 4 * n - 8;
                t = up ? b - 1 : b + 1;
                if (t < 0 || t >= B) {
                    T[b * nc + j] = 0u;
                    continue;
                }
                D = (lnW[t] - lnW[b]) - c->beta * (double)dE;
            }
            T[b * nc + j] = threshold(D);
        }
}

static int accept(uint32_t T, uint32_t r)
{
    return T == 0xffffffffu || r < T;
}

/* Run n_sweeps sweeps (global sweep ids g0, g0+1, ...) of chains
 * [ch_lo, ch_hi).  A sweep visits sites 0..N-1 in row-major order; after each
 * sweep the chain's bin is added to H if record != 0.  E and M are carried. */
static int sweeps_impl(const orc_lattice *c, int8_t *spins, int32_t *E, int32_t *M,
                       const uint32_t *T, uint32_t g0, int64_t n_sweeps, int record,
                       uint64_t *H, uint64_t *HEM, uint64_t *ACC, int32_t ch_lo, int32_t ch_hi)
{
    int32_t L = c->L, N = L * L, nc = orc_ncols(c->model), B = orc_nbins(c);
    int32_t step = bin_step(c->model), ch;
    for (ch = ch_lo; ch < ch_hi; ++ch) {
        int8_t *s = spins + (int64_t)ch * N;
        int64_t sw;
        for (sw = 0; sw < n_sweeps; ++sw) {
            uint32_t g = g0 + (uint32_t)sw;
            uint32_t w[4];
            int32_t i, b;
            for (i = 0; i < N; ++i) {
                int32_t y = i / L, x = i % L;
                int32_t nb[4];
                nb[0] = s[site(L, y, x + 1)];
                nb[1] = s[site(L, y, x - 1)];
                nb[2] = s[site(L, y + 1, x)];
                nb[3] = s[site(L, y - 1, x)];
                if (c->model == ORC_POTTS) {
                    /* colours 0..q-1 (q <= 255) are stored as unsigned bytes */
                    uint32_t wp, wa;
                    int32_t old = (uint8_t)s[i], nw, n_old = 0, n_new = 0, k, dE;
                    for (k = 0; k < 4; ++k)
                        nb[k] = (uint8_t)nb[k];
                    if ((i & 1) == 0)
                        draw(c->seed, (uint32_t)ch, g, (uint32_t)(i >> 1), ORC_TAG_SWEEP, w);
                    wp = w[2 * (i & 1)];
                    wa = w[2 * (i & 1) + 1];
                    /* proposal: one of the q-1 other colours, uniformly */
                    nw = (old + 1 + (int32_t)(((uint64_t)wp * (uint64_t)(c->q - 1)) >> 32)) % c->q;
                    for (k = 0; k < 4; ++k) {
                        n_old += (nb[k] == old);
                        n_new += (nb[k] == nw);
                    }
                    dE = n_old - n_new; /* change of unsatisfied bonds */
                    b = (E[ch] - c->lo) / step;
                    if (accept(T[b * nc + (dE + 4)], wa)) {
                        s[i] = (int8_t)nw;
                        E[ch] += dE;
                        if (record && ACC)
                            *ACC += 1u;
                    }
                } else {
                    uint32_t r;
                    int32_t sum = nb[0] + nb[1] + nb[2] + nb[3];
                    int32_t dE = 2 * s[i] * sum; /* flip s_i -> -s_i */
                    int32_t n_al = (s[i] * sum + 4) / 2;
                    if ((i & 3) == 0)
                        draw(c->seed, (uint32_t)ch, g, (uint32_t)(i >> 2), ORC_TAG_SWEEP, w);
                    r = w[i & 3];
                    if (c->model == ORC_ISING) {
                        b = (E[ch] - c->lo) / step;
                        if (accept(T[b * nc + n_al], r)) {
                            s[i] = (int8_t)(-s[i]);
                            E[ch] += dE;
                            M[ch] += 2 * s[i];
                            if (record && ACC)
                                *ACC += 1u;
                        }
                    } else {
                        b = (M[ch] - c->lo) / step;
                        if (accept(T[b * nc + 2 * n_al + (s[i] > 0)], r)) {
                            s[i] = (int8_t)(-s[i]);
                            E[ch] += dE;
                            M[ch] += 2 * s[i];
                            if (record && ACC)
                                *ACC += 1u;
                        }
                    }
                }
            }
            if (record) {
                int32_t v = (c->model == ORC_MUMA) ? M[ch] : E[ch];
                b = (v - c->lo) / step;
                if (b < 0 || b >= B)
                    return -1;
                H[b] += 1u;
                if (HEM) {
                    /* E = -2N + 4e, e = 0..N: the row of the joint histogram */
                    int32_t e = (E[ch] + 2 * N) / 4;
                    HEM[(int64_t)e * B + b] += 1u;
                }
            }
        }
    }
    return 0;
}

int orc_sweeps(const orc_lattice *c, int8_t *spins, int32_t *E, int32_t *M,
               const uint32_t *T, uint32_t g0, int64_t n_sweeps, int record,
               uint64_t *H, int32_t ch_lo, int32_t ch_hi)
{
    return sweeps_impl(c, spins, E, M, T, g0, n_sweeps, record, H, NULL, NULL, ch_lo, ch_hi);
}

/* orc_sweeps that also adds the number of accepted moves of the recorded
 * sweeps to *ACC (the acceptance rate of an iteration). */
int orc_sweeps_acc(const orc_lattice *c, int8_t *spins, int32_t *E, int32_t *M,
                   const uint32_t *T, uint32_t g0, int64_t n_sweeps, int record,
                   uint64_t *H, uint64_t *ACC, int32_t ch_lo, int32_t ch_hi)
{
    return sweeps_impl(c, spins, E, M, T, g0, n_sweeps, record, H, NULL, ACC, ch_lo, ch_hi);
}

/* orc_sweeps of a MUMA run that also counts every recorded sweep in
 * HEM[e * B + b] (e = (E + 2N) / 4, b = the magnetisation bin), the state
 * after the sweep.  -2 if the run is not multimagnetic. */
int orc_sweeps_em(const orc_lattice *c, int8_t *spins, int32_t *E, int32_t *M,
                  const uint32_t *T, uint32_t g0, int64_t n_sweeps, int record,
                  uint64_t *H, uint64_t *HEM, int32_t ch_lo, int32_t ch_hi)
{
    if (c->model != ORC_MUMA)
        return -2;
    return sweeps_impl(c, spins, E, M, T, g0, n_sweeps, record, H, HEM, NULL, ch_lo, ch_hi);
}

/* ------------------------------------------------------------------------ */
/* Weight recursion with accumulated statistics, in log weights.            */
/*                                                                          */
/* lnR[k] = lnW(r_{k+1}) - lnW(r_k) over consecutive reachable bins r_k.     */
/* Iteration n measures, for each pair, ln H(r_k) - ln H(r_{k+1}) + lnR^(n) */
/* as an estimate of -(ln Omega(r_{k+1}) - ln Omega(r_k)), with variance     */
/* ~ 1/H(r_k) + 1/H(r_{k+1}) = 1/p.  The inverse-variance-weighted mean over */
/* all iterations so far, written recursively, is                            */
/*   P[k] += p;  lnR[k] += (p / P[k]) * (ln H(r_k) - ln H(r_{k+1})),         */
/* with p = H(r_k) H(r_{k+1}) / (H(r_k) + H(r_{k+1})) and p = 0 if either    */
/* bin is empty.  With no earlier statistics p/P = 1 and this is            */
/* W^(n+1) = W^(n) / H^(n).  lnW(r_0) = 0; a bin that is never reachable    */
/* carries the weight of the reachable bin below it (or of r_0).            */
/* lnR and P are indexed by the lower bin of each pair (size B).            */
/* ------------------------------------------------------------------------ */
void orc_recursion(int32_t B, const uint8_t *mask, const uint64_t *H, double *lnR,
                   double *P, double *lnW)
{
    int32_t b, prev = -1;
    for (b = 0; b < B; ++b) {
        if (!mask[b])
            continue;
        if (prev >= 0) {
            double h0 = (double)H[prev], h1 = (double)H[b];
            double p = 0.0;
            if (H[prev] > 0 && H[b] > 0)
                p = (h0 * h1) / (h0 + h1);
            P[prev] = P[prev] + p;
            if (p > 0.0) {
                double kappa = p / P[prev];
                lnR[prev] = lnR[prev] + kappa * (log(h0) - log(h1));
            }
        }
        prev = b;
    }
    /* rebuild lnW by the cumulative sum over the reachable sequence */
    {
        double acc = 0.0;
        int32_t last = -1;
        for (b = 0; b < B; ++b) {
            if (mask[b]) {
                if (last >= 0)
                    acc = acc + lnR[last];
                last = b;
            }
            lnW[b] = acc;
        }
    }
}

/* min over reachable bins / mean over reachable bins of H */
double orc_flatness(int32_t B, const uint8_t *mask, const uint64_t *H)
{
    int32_t b, n = 0;
    double sum = 0.0, mn = 0.0;
    for (b = 0; b < B; ++b) {
        if (!mask[b])
            continue;
        if (n == 0 || (double)H[b] < mn)
            mn = (double)H[b];
        sum += (double)H[b];
        ++n;
    }
    if (n == 0 || sum <= 0.0)
        return 0.0;
    return mn / (sum / (double)n);
}

/* ------------------------------------------------------------------------ */
/* Reweighting, Eq. 2, over the histogram of the binned quantity.            */
/* value[b] is the physical value of bin b (energy, or M for MUMA).          */
/* Energy ensembles: a_b = ln H_b - lnW_b - beta E_b; w_b = exp(a_b - max a);*/
/*   out = { <E>/Nsite, beta^2 Var(E)/Nsite, <E>, max a + ln sum w }.        */
/* MUMA (canonical at the simulation beta): a_b = ln H_b - lnW_b;            */
/*   out = { <|M|>/Nsite, <M^2>/Nsite^2, <M>/Nsite, max a + ln sum w }.      */
/* Sums run in ascending bin order.                                          */
/* ------------------------------------------------------------------------ */
void orc_reweight(int32_t B, const uint64_t *H, const double *lnW, const double *value,
                  int32_t nsite, int32_t muma, double beta, double *out)
{
    int32_t b, any = 0;
    double amax = 0.0, Z = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (b = 0; b < B; ++b) {
        double a;
        if (H[b] == 0)
            continue;
        a = log((double)H[b]) - lnW[b];
        if (!muma)
            a = a - beta * value[b];
        if (!any || a > amax)
            amax = a;
        any = 1;
    }
    if (!any) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    for (b = 0; b < B; ++b) {
        double a, w;
        if (H[b] == 0)
            continue;
        a = log((double)H[b]) - lnW[b];
        if (!muma)
            a = a - beta * value[b];
        w = exp(a - amax);
        Z += w;
        if (muma) {
            m1 += w * fabs(value[b]);
            m2 += w * (value[b] * value[b]);
            m3 += w * value[b];
        } else {
            m1 += w * value[b];
        }
    }
    if (muma) {
        double n = (double)nsite;
        out[0] = (m1 / Z) / n;
        out[1] = (m2 / Z) / (n * n);
        out[2] = (m3 / Z) / n;
        out[3] = amax + log(Z);
        return;
    }
    {
        double mean = m1 / Z, var = 0.0;
        for (b = 0; b < B; ++b) {
            double a, w, d;
            if (H[b] == 0)
                continue;
            a = log((double)H[b]) - lnW[b] - beta * value[b];
            w = exp(a - amax);
            d = value[b] - mean;
            var += w * (d * d);
        }
        var = var / Z;
        out[0] = mean / (double)nsite;
        out[1] = (beta * beta) * var / (double)nsite;
        out[2] = mean;
        out[3] = amax + log(Z);
    }
}

/* ------------------------------------------------------------------------ */
/* Reweighting of a multimagnetic run to the canonical ensemble at beta2.    */
/* The run samples states with weight exp(-beta E) W(M) (Eq. 3); the         */
/* canonical weight at beta2 relative to that is exp(-(beta2 - beta) E)/W(M),*/
/* so over the joint histogram HEM[e][b] (E_e = Ev[e], M_b = Mv[b]):         */
/*   a = ln HEM[e][b] - lnW[b] - (beta2 - beta) E_e,  w = exp(a - max a),    */
/*   out = { <E>/N, beta2^2 Var(E)/N, <|M|>/N, <M^2>/N^2,                   */
/*           beta2 (<M^2> - <|M|>^2)/N, max a + ln sum w }.                  */
/* Sums run over e, then b, ascending; the variance of E is a second pass    */
/* around the mean.                                                          */
/* ------------------------------------------------------------------------ */
void orc_reweight_em(int32_t NE, int32_t B, const uint64_t *HEM, const double *lnW, const double *Ev,
                     const double *Mv, int32_t nsite, double beta, double beta2, double *out)
{
    int32_t e, b, any = 0;
    double amax = 0.0, Z = 0.0, s_e = 0.0, s_am = 0.0, s_m2 = 0.0, mean, var = 0.0, n = (double)nsite;
    for (e = 0; e < NE; ++e)
        for (b = 0; b < B; ++b) {
            double a;
            if (HEM[(int64_t)e * B + b] == 0)
                continue;
            a = log((double)HEM[(int64_t)e * B + b]) - lnW[b] - (beta2 - beta) * Ev[e];
            if (!any || a > amax)
                amax = a;
            any = 1;
        }
    if (!any) {
        for (e = 0; e < 6; ++e)
            out[e] = 0.0;
        return;
    }
    for (e = 0; e < NE; ++e)
        for (b = 0; b < B; ++b) {
            double a, w;
            if (HEM[(int64_t)e * B + b] == 0)
                continue;
            a = log((double)HEM[(int64_t)e * B + b]) - lnW[b] - (beta2 - beta) * Ev[e];
            w = exp(a - amax);
            Z += w;
            s_e += w * Ev[e];
            s_am += w * fabs(Mv[b]);
            s_m2 += w * (Mv[b] * Mv[b]);
        }
    mean = s_e / Z;
    for (e = 0; e < NE; ++e)
        for (b = 0; b < B; ++b) {
            double a, w, d;
            if (HEM[(int64_t)e * B + b] == 0)
                continue;
            a = log((double)HEM[(int64_t)e * B + b]) - lnW[b] - (beta2 - beta) * Ev[e];
            w = exp(a - amax);
            d = Ev[e] - mean;
            var += w * (d * d);
        }
    var = var / Z;
    out[0] = mean / n;
    out[1] = beta2 * beta2 * var / n;
    out[2] = (s_am / Z) / n;
    out[3] = (s_m2 / Z) / (n * n);
    out[4] = beta2 * ((s_m2 / Z) - (s_am / Z) * (s_am / Z)) / n;
    out[5] = amax + log(Z);
}

/* ------------------------------------------------------------------------ */
/* Bead-spring homopolymer (Eq. 7) with single-monomer shift moves.          */
/*                                                                          */
/* Pair potential on |i-j| >= 2: Lennard-Jones 4 eps [(sig/r)^12-(sig/r)^6]  */
/* cut at r_c and shifted to zero there.  Bonds |i-j| = 1: FENE in the       */
/* paper's form -(K/2) R^2 ln(1 - ((r - r0)/R)^2), infinite (move rejected)  */
/* when |r - r0| >= R.  Positions are float; energies double.               */
/* Move of bead i in sweep g uses one Philox call (chain, g, i, SWEEP):      */
/* words 0..2 give the displacement ((w>>8) 2^-24 - 1/2) * step per axis,    */
/* word 3 is the acceptance word.                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_beads;
    int32_t n_chains;
    uint64_t seed;
    double x_lo, x_hi; /* energy range [x_lo, x_hi)                      */
    int32_t n_bins;
    double lj_eps, lj_sigma, lj_rcut;
    double fene_k, fene_r0, fene_R;
    float step;        /* side of the displacement cube                  */
    int32_t moves;     /* 0: shifts; 1: shifts, spherical rotations and   */
                       /* double bridging (the paper's move set)          */
} orc_polymer;

static double lj_shift(const orc_polymer *p)
{
    double sr2 = (p->lj_sigma * p->lj_sigma) / (p->lj_rcut * p->lj_rcut);
    double sr6 = sr2 * sr2 * sr2;
    return 4.0 * p->lj_eps * (sr6 * sr6 - sr6);
}

/* FENE bond energy at squared length r2; 0 and *broken = 1 outside the
 * bond's domain */
static double fene(const orc_polymer *p, double r2, int *broken)
{
    double r = sqrt(r2);
    double t = (r - p->fene_r0) / p->fene_R;
    double arg = 1.0 - t * t;
    if (!(arg > 0.0)) {
        *broken = 1;
        return 0.0;
    }
    return -(0.5 * p->fene_k * p->fene_R * p->fene_R) * log(arg);
}

/* cut and shifted Lennard-Jones energy at squared distance r2 */
static double lj(const orc_polymer *p, double r2)
{
    if (r2 < p->lj_rcut * p->lj_rcut) {
        double sr2 = (p->lj_sigma * p->lj_sigma) / r2;
        double sr6 = sr2 * sr2 * sr2;
        return 4.0 * p->lj_eps * (sr6 * sr6 - sr6) - lj_shift(p);
    }
    return 0.0;
}

/* energy of one pair at squared distance r2; returns 0 if a bond is broken
 * (and sets *broken) */
static double pair_energy(const orc_polymer *p, int32_t i, int32_t j, double r2, int *broken)
{
    int32_t sep = i > j ? i - j : j - i;
    if (sep == 1)
        return fene(p, r2, broken);
    return lj(p, r2);
}

static double dist2(const float *a, const float *b)
{
    double dx = (double)a[0] - (double)b[0];
    double dy = (double)a[1] - (double)b[1];
    double dz = (double)a[2] - (double)b[2];
    return dx * dx + dy * dy + dz * dz;
}

/* total energy of one chain (pos[bead][3]); pairs i<j in ascending order */
double orc_polymer_energy(const orc_polymer *p, const float *pos, int *broken)
{
    int32_t i, j;
    double e = 0.0;
    *broken = 0;
    for (i = 0; i < p->n_beads; ++i)
        for (j = i + 1; j < p->n_beads; ++j)
            e += pair_energy(p, i, j, dist2(pos + 3 * i, pos + 3 * j), broken);
    return e;
}

/* bin of energy E, or -1 outside [x_lo, x_hi) */
int32_t orc_polymer_bin(const orc_polymer *p, double E)
{
    double scale = (double)p->n_bins / (p->x_hi - p->x_lo);
    double f;
    if (!(E >= p->x_lo) || !(E < p->x_hi))
        return -1;
    f = floor((E - p->x_lo) * scale);
    if (f < 0.0)
        return -1;
    if (f >= (double)p->n_bins)
        return -1;
    return (int32_t)f;
}

/* pos[chain][bead][3]; E[chain] and bin[chain] are outputs */
int orc_polymer_init(const orc_polymer *p, const float *pos, double *E, int32_t *bin)
{
    int32_t ch;
    for (ch = 0; ch < p->n_chains; ++ch) {
        int broken = 0;
        E[ch] = orc_polymer_energy(p, pos + (int64_t)ch * p->n_beads * 3, &broken);
        bin[ch] = broken ? -1 : orc_polymer_bin(p, E[ch]);
        if (bin[ch] < 0)
            return -1;
    }
    return 0;
}

/* the new-minus-old energy of the pair (i, j) when bead i moves to xn */
static double pair_delta(const orc_polymer *p, const float *pos, int32_t i, int32_t j,
                         const float *xn, int *broken)
{
    double en, eo;
    if (j >= p->n_beads || j == i)
        return 0.0;
    en = pair_energy(p, i, j, dist2(xn, pos + 3 * j), broken);
    eo = pair_energy(p, i, j, dist2(pos + 3 * i, pos + 3 * j), broken);
    return en - eo;
}

/* dE of moving bead i to xn: per-partner terms summed by a fixed binary
 * tree over 64 slots (slot j holds partner j's term, zero for j == i and
 * j >= n_beads; for n_beads > 64 slot j holds partner j's term plus partner
 * j + 64's term): for stride 32, 16, ..., 1, slot k += slot k + stride. */
static double polymer_delta(const orc_polymer *p, const float *pos, int32_t i,
                            const float *xn, int *broken)
{
    double t[64];
    int32_t j, stride;
    for (j = 0; j < 64; ++j) {
        t[j] = pair_delta(p, pos, i, j, xn, broken);
        if (p->n_beads > 64)
            t[j] = t[j] + pair_delta(p, pos, i, j + 64, xn, broken);
    }
    for (stride = 32; stride >= 1; stride /= 2)
        for (j = 0; j < stride; ++j)
            t[j] = t[j] + t[j + stride];
    return t[0];
}

/* Spherical rotation of bead i (the paper names the move; its form here):
 * an inner bead turns about the line through its two neighbours, an end
 * bead about a coordinate axis (chosen by word 1) through its neighbour, so
 * every bond length is kept.  The rotation is that of the quaternion
 * (tau, a), a the axis direction, not normalised: angle 2 atan2(|a|, tau).
 * tau comes from word 0: u = (k - (2^23 - 1/2)) / 2^23 in (-1, 1) for
 * k = w >> 8, tau = u / (1 - |u|), so tau and -tau (the inverse rotation)
 * are equally likely and the proposal is symmetric.  Only +, -, *, / in
 * double, in the order written, then one rounding to float per axis. */
static double rot_tau(uint32_t w)
{
    double u = ((double)(w >> 8) - 8388607.5) / 8388608.0;
    return u / (1.0 - fabs(u));
}

static void quat_rotate(double w, const double a[3], const double v[3], double out[3])
{
    double x = a[0], y = a[1], z = a[2];
    double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    double n2 = ((ww + xx) + yy) + zz;
    double m00 = ((ww + xx) - yy) - zz, m11 = ((ww - xx) + yy) - zz, m22 = ((ww - xx) - yy) + zz;
    double m01 = 2.0 * (x * y - w * z), m02 = 2.0 * (x * z + w * y);
    double m10 = 2.0 * (x * y + w * z), m12 = 2.0 * (y * z - w * x);
    double m20 = 2.0 * (x * z - w * y), m21 = 2.0 * (y * z + w * x);
    out[0] = ((m00 * v[0] + m01 * v[1]) + m02 * v[2]) / n2;
    out[1] = ((m10 * v[0] + m11 * v[1]) + m12 * v[2]) / n2;
    out[2] = ((m20 * v[0] + m21 * v[1]) + m22 * v[2]) / n2;
}

static void rotation_proposal(const orc_polymer *p, const float *x, int32_t i, const uint32_t w[4],
                              float xn[3])
{
    int32_t nb = p->n_beads, k, ctr;
    double a[3], v[3], r[3], c[3];
    if (i > 0 && i < nb - 1) {
        ctr = i - 1;
        for (k = 0; k < 3; ++k)
            a[k] = (double)x[3 * (i + 1) + k] - (double)x[3 * (i - 1) + k];
    } else {
        uint32_t ax = (uint32_t)(((uint64_t)w[1] * 3u) >> 32);
        ctr = i == 0 ? 1 : nb - 2;
        for (k = 0; k < 3; ++k)
            a[k] = (uint32_t)k == ax ? 1.0 : 0.0;
    }
    for (k = 0; k < 3; ++k) {
        c[k] = (double)x[3 * ctr + k];
        v[k] = (double)x[3 * i + k] - c[k];
    }
    quat_rotate(rot_tau(w[0]), a, v, r);
    for (k = 0; k < 3; ++k)
        xn[k] = (float)(c[k] + r[k]);
}

/* Double bridging (the paper names the move; its form here): bonds (i, i+1)
 * and (j, j+1), i + 2 <= j, are replaced by (i, j) and (i+1, j+1) and the
 * beads i+1 .. j are renumbered in reverse, so the chain stays linear and
 * no bead moves.  i and j come from words 0 and 1 (uniform in 0 .. N-2,
 * ordered; pairs closer than 2 do nothing); the move is its own inverse.
 * Energy change: the four bonds swap between FENE and LJ:
 *   dE = ((F(ij) + F(i+1,j+1)) - F(i,i+1)) - F(j,j+1)
 *      + ((L(i,i+1) + L(j,j+1)) - L(ij)) - L(i+1,j+1).
 * Returns 1 and sets *dE, *pi, *pj for a proposal, 0 for none or a new bond
 * outside the FENE domain. */
static int bridging_proposal(const orc_polymer *p, const float *x, const uint32_t w[4], double *dE,
                             int32_t *pi, int32_t *pj)
{
    int32_t nb = p->n_beads, i, j, t;
    int broken = 0;
    double fij, fkl, fik, fjl, lij, lkl, lik, ljl, dF, dL;
    if (nb < 4)
        return 0;
    i = (int32_t)(((uint64_t)w[0] * (uint64_t)(nb - 1)) >> 32);
    j = (int32_t)(((uint64_t)w[1] * (uint64_t)(nb - 1)) >> 32);
    if (i > j) {
        t = i;
        i = j;
        j = t;
    }
    if (j - i < 2)
        return 0;
    /* new bonds (i, j), (i+1, j+1); old bonds (i, i+1), (j, j+1) */
    fij = fene(p, dist2(x + 3 * i, x + 3 * j), &broken);
    fkl = fene(p, dist2(x + 3 * (i + 1), x + 3 * (j + 1)), &broken);
    if (broken)
        return 0;
    fik = fene(p, dist2(x + 3 * i, x + 3 * (i + 1)), &broken);
    fjl = fene(p, dist2(x + 3 * j, x + 3 * (j + 1)), &broken);
    lij = lj(p, dist2(x + 3 * i, x + 3 * j));
    lkl = lj(p, dist2(x + 3 * (i + 1), x + 3 * (j + 1)));
    lik = lj(p, dist2(x + 3 * i, x + 3 * (i + 1)));
    ljl = lj(p, dist2(x + 3 * j, x + 3 * (j + 1)));
    dF = ((fij + fkl) - fik) - fjl;
    dL = ((lik + ljl) - lij) - lkl;
    *dE = dF + dL;
    *pi = i;
    *pj = j;
    return 1;
}

/* test hooks: the proposals of one chain (pos[bead][3]) */
void orc_polymer_rotation(const orc_polymer *p, const float *pos, int32_t i, const uint32_t w[4], float xn[3])
{
    rotation_proposal(p, pos, i, w, xn);
}

int orc_polymer_bridging(const orc_polymer *p, const float *pos, const uint32_t w[4], double *dE, int32_t *i,
                         int32_t *j)
{
    return bridging_proposal(p, pos, w, dE, i, j);
}

/* MUCA acceptance of a proposal with energy change dE for chain ch; on
 * acceptance E and the bin advance */
static int polymer_accept(const orc_polymer *p, const double *lnW, double *E, int32_t *bin, double dE,
                          uint32_t word)
{
    double En = *E + dE;
    int32_t bn = orc_polymer_bin(p, En);
    if (bn < 0)
        return 0;
    if (!accept(threshold(lnW[bn] - lnW[*bin]), word))
        return 0;
    *E = En;
    *bin = bn;
    return 1;
}

/* T2 is the B x B threshold matrix T2[b*B + b'] of lnW(b') - lnW(b); pass
 * NULL to evaluate the rule from lnW directly (same values). */
int orc_polymer_sweeps_acc(const orc_polymer *p, float *pos, double *E, int32_t *bin,
                           const double *lnW, uint32_t g0, int64_t n_sweeps, int record,
                           uint64_t *H, uint64_t *ACC, int32_t ch_lo, int32_t ch_hi);

int orc_polymer_sweeps(const orc_polymer *p, float *pos, double *E, int32_t *bin,
                       const double *lnW, uint32_t g0, int64_t n_sweeps, int record,
                       uint64_t *H, int32_t ch_lo, int32_t ch_hi)
{
    return orc_polymer_sweeps_acc(p, pos, E, bin, lnW, g0, n_sweeps, record, H, NULL, ch_lo, ch_hi);
}

/* orc_polymer_sweeps that also adds the accepted moves of the recorded
 * sweeps to *ACC. */
int orc_polymer_sweeps_acc(const orc_polymer *p, float *pos, double *E, int32_t *bin,
                           const double *lnW, uint32_t g0, int64_t n_sweeps, int record,
                           uint64_t *H, uint64_t *ACC, int32_t ch_lo, int32_t ch_hi)
{
    int32_t ch, nb = p->n_beads;
    for (ch = ch_lo; ch < ch_hi; ++ch) {
        float *x = pos + (int64_t)ch * nb * 3;
        int64_t sw;
        for (sw = 0; sw < n_sweeps; ++sw) {
            uint32_t g = g0 + (uint32_t)sw;
            int32_t i;
            for (i = 0; i < nb; ++i) {
                uint32_t w[4];
                float xn[3];
                int k, broken = 0;
                double dE, En;
                int32_t bn;
                draw(p->seed, (uint32_t)ch, g, (uint32_t)i, ORC_TAG_SWEEP, w);
                for (k = 0; k < 3; ++k) {
                    float u = (float)(w[k] >> 8) * 5.9604644775390625e-08f; /* 2^-24 */
                    float d = (u - 0.5f) * p->step;
                    xn[k] = x[3 * i + k] + d;
                }
                dE = polymer_delta(p, x, i, xn, &broken);
                if (broken)
                    continue;
                En = E[ch] + dE;
                bn = orc_polymer_bin(p, En);
                if (bn < 0)
                    continue;
                if (accept(threshold(lnW[bn] - lnW[bin[ch]]), w[3])) {
                    x[3 * i + 0] = xn[0];
                    x[3 * i + 1] = xn[1];
                    x[3 * i + 2] = xn[2];
                    E[ch] = En;
                    bin[ch] = bn;
                    if (record && ACC)
                        *ACC += 1u;
                }
            }
            if (p->moves) {
                int32_t bi, bj, k;
                double dEb;
                /* a spherical rotation of every bead, in order */
                for (i = 0; i < nb; ++i) {
                    uint32_t w[4];
                    float xn[3];
                    int broken = 0;
                    double dE;
                    draw(p->seed, (uint32_t)ch, g, (uint32_t)i, ORC_TAG_ROT, w);
                    rotation_proposal(p, x, i, w, xn);
                    dE = polymer_delta(p, x, i, xn, &broken);
                    if (broken)
                        continue;
                    if (polymer_accept(p, lnW, &E[ch], &bin[ch], dE, w[3])) {
                        x[3 * i + 0] = xn[0];
                        x[3 * i + 1] = xn[1];
                        x[3 * i + 2] = xn[2];
                        if (record && ACC)
                            *ACC += 1u;
                    }
                }
                /* one double-bridging attempt */
                {
                    uint32_t w[4];
                    draw(p->seed, (uint32_t)ch, g, 0u, ORC_TAG_BRIDGE, w);
                    if (bridging_proposal(p, x, w, &dEb, &bi, &bj) &&
                        polymer_accept(p, lnW, &E[ch], &bin[ch], dEb, w[3])) {
                        if (record && ACC)
                            *ACC += 1u;
                        for (i = bi + 1, k = bj; i < k; ++i, --k) {
                            int32_t d;
                            for (d = 0; d < 3; ++d) {
                                float tmp = x[3 * i + d];
                                x[3 * i + d] = x[3 * k + d];
                                x[3 * k + d] = tmp;
                            }
                        }
                    }
                }
            }
            if (record)
                H[bin[ch]] += 1u;
        }
    }
    return 0;
}
