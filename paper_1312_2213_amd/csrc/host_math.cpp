// host_math.cpp -- the host-side FP64 arithmetic of the multicanonical
// iteration (see host_math.h).  Every sum runs in ascending bin order with
// glibc's log and exp, so its results are reproducible bit for bit.
#include "host_math.h"

#include <cmath>

#include "../../include/muca.h"

// Values of the binned quantity that no lattice configuration takes
// (Omega = 0 on the even-L torus): Ising E = +-(2N - 4); Potts q = 2 odd
// E_unsat and E_unsat in {2, 2N - 2}; Potts q >= 3 E_unsat in {1, 2, 3, 5}.
// The recursion links consecutive bins of the remaining set and flatness is
// measured over it.
void muca_reachable_mask(int model, int q, int lo, int step, int n_sites, int n_bins, uint8_t *m)
{
    const int N = n_sites;
    for (int b = 0; b < n_bins; ++b) {
        m[b] = 1;
        const int v = lo + b * step;
        if (model == MUCA_ISING) {
            if (v == 2 * N - 4 || v == -(2 * N - 4))
                m[b] = 0;
        } else if (model == MUCA_POTTS) {
            if (q == 2) {
                if ((v % 2) != 0 || v == 2 || v == 2 * N - 2)
                    m[b] = 0;
            } else if (v == 1 || v == 2 || v == 3 || v == 5) {
                m[b] = 0;
            }
        }
    }
}

uint32_t muca_threshold_of(double D)
{
    if (D >= 0.0)
        return 0xffffffffu;
    // 2^32 e^D < 1 for D < -32 ln 2 = -22.18: the threshold is 0, no exp needed
    if (D < -23.0)
        return 0u;
    const double v = std::exp(D) * 4294967296.0; // times 2^32: exact
    if (v >= 4294967295.0)
        return 0xffffffffu;
    return (uint32_t)std::floor(v);
}

void muca_lattice_thresholds(int model, double beta, int n_bins, int n_cols, const double *lnW, uint32_t *T)
{
    const int B = n_bins, NC = n_cols;
    for (int b = 0; b < B; ++b) {
        for (int j = 0; j < NC; ++j) {
            int target;
            double D;
            if (model == MUCA_ISING) {
                target = b + j - 2; // column = aligned neighbours, dE = 4j - 8
            } else if (model == MUCA_POTTS) {
                target = b + j - 4; // column = dE_unsat + 4
            } else {
                target = (j & 1) ? b - 1 : b + 1; // column = 2 n_aligned + (s_i == +1)
            }
            if (target < 0 || target >= B) {
                T[(size_t)b * NC + j] = 0u;
                continue;
            }
            D = lnW[target] - lnW[b];
            if (model == MUCA_MUMA) {
                const int dE = 4 * (j >> 1) - 8;
                D = D - beta * (double)dE;
            }
            T[(size_t)b * NC + j] = muca_threshold_of(D);
        }
    }
}

// ---------------------------------------------------------------------------
// Accumulated-statistics recursion on consecutive bins of the set `m`:
//   p = h0 h1 / (h0 + h1) (0 if a bin is empty),  P += p,
//   lnR += (p / P) (ln h0 - ln h1),
// then lnW is the running sum of lnR from the first bin of the set (lnW = 0
// there); bins outside the set repeat the last weight.
// ---------------------------------------------------------------------------
void muca_recursion(int B, const uint8_t *m, const uint64_t *H, double *lnR, double *P, double *lnW)
{
    int lower = -1;
    for (int b = 0; b < B; ++b) {
        if (!m[b])
            continue;
        if (lower >= 0) {
            const uint64_t a = H[lower], c = H[b];
            double p = 0.0;
            if (a != 0 && c != 0) {
                const double h0 = (double)a, h1 = (double)c;
                p = (h0 * h1) / (h0 + h1);
            }
            P[lower] = P[lower] + p;
            if (p > 0.0) {
                const double kappa = p / P[lower];
                lnR[lower] = lnR[lower] + kappa * (std::log((double)a) - std::log((double)c));
            }
        }
        lower = b;
    }
    double run = 0.0;
    int last = -1;
    for (int b = 0; b < B; ++b) {
        if (m[b]) {
            if (last >= 0)
                run = run + lnR[last];
            last = b;
        }
        lnW[b] = run;
    }
}

double muca_flatness(int B, const uint8_t *m, const uint64_t *H)
{
    double lo = 0.0, sum = 0.0;
    int n = 0;
    for (int b = 0; b < B; ++b) {
        if (!m[b])
            continue;
        const double h = (double)H[b];
        if (n == 0 || h < lo)
            lo = h;
        sum += h;
        ++n;
    }
    if (n == 0 || sum <= 0.0)
        return 0.0;
    return lo / (sum / (double)n);
}

// Reweighting, Eq. 2, on the binned histogram.  Sums in ascending bin order.
void muca_reweight_bins(int B, const uint64_t *H, const double *lnW, const double *val, int nsite,
                        bool muma, double beta, double *out)
{
    double amax = 0.0;
    bool any = false;
    for (int b = 0; b < B; ++b) {
        if (!H[b])
            continue;
        double a = std::log((double)H[b]) - lnW[b];
        if (!muma)
            a = a - beta * val[b];
        if (!any || a > amax)
            amax = a;
        any = true;
    }
    if (!any) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    double Z = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int b = 0; b < B; ++b) {
        if (!H[b])
            continue;
        double a = std::log((double)H[b]) - lnW[b];
        if (!muma)
            a = a - beta * val[b];
        const double w = std::exp(a - amax);
        Z += w;
        if (muma) {
            s1 += w * std::fabs(val[b]);
            s2 += w * (val[b] * val[b]);
            s3 += w * val[b];
        } else {
            s1 += w * val[b];
        }
    }
    const double n = (double)nsite;
    if (muma) {
        out[0] = (s1 / Z) / n;
        out[1] = (s2 / Z) / (n * n);
        out[2] = (s3 / Z) / n;
        out[3] = amax + std::log(Z);
        return;
    }
    const double mean = s1 / Z;
    double var = 0.0;
    for (int b = 0; b < B; ++b) {
        if (!H[b])
            continue;
        const double a = std::log((double)H[b]) - lnW[b] - beta * val[b];
        const double w = std::exp(a - amax);
        const double d = val[b] - mean;
        var += w * (d * d);
    }
    var = var / Z;
    out[0] = mean / n;
    out[1] = (beta * beta) * var / n;
    out[2] = mean;
    out[3] = amax + std::log(Z);
}


// Each state's canonical weight at beta2 relative to its sampling weight
// exp(-beta E) W(M) is exp(-(beta2 - beta) E) / W(M).
void muca_reweight_joint(int NE, int B, const uint64_t *h, const double *lnW, int32_t lo, int32_t mstep, int nsite,
                         double beta, double beta2, double *out)
{
    auto energy = [&](int e) { return -2.0 * nsite + 4.0 * e; };
    auto magnet = [&](int b) { return (double)lo + (double)mstep * b; };
    auto log_w = [&](int e, int b) {
        return std::log((double)h[(size_t)e * B + b]) - lnW[b] - (beta2 - beta) * energy(e);
    };
    double amax = 0.0;
    bool any = false;
    for (int e = 0; e < NE; ++e)
        for (int b = 0; b < B; ++b)
            if (h[(size_t)e * B + b]) {
                const double a = log_w(e, b);
                if (!any || a > amax)
                    amax = a;
                any = true;
            }
    if (!any) {
        for (int k = 0; k < 6; ++k)
            out[k] = 0.0;
        return;
    }
    double Z = 0.0, sE = 0.0, sA = 0.0, s2 = 0.0;
    for (int e = 0; e < NE; ++e)
        for (int b = 0; b < B; ++b)
            if (h[(size_t)e * B + b]) {
                const double w = std::exp(log_w(e, b) - amax), m = magnet(b);
                Z += w;
                sE += w * energy(e);
                sA += w * std::fabs(m);
                s2 += w * (m * m);
            }
    const double mean = sE / Z;
    double var = 0.0;
    for (int e = 0; e < NE; ++e)
        for (int b = 0; b < B; ++b)
            if (h[(size_t)e * B + b]) {
                const double w = std::exp(log_w(e, b) - amax), d = energy(e) - mean;
                var += w * (d * d);
            }
    var /= Z;
    const double n = (double)nsite, mA = sA / Z, m2 = s2 / Z;
    out[0] = mean / n;
    out[1] = beta2 * beta2 * var / n;
    out[2] = mA / n;
    out[3] = m2 / (n * n);
    out[4] = beta2 * (m2 - mA * mA) / n;
    out[5] = amax + std::log(Z);
}
