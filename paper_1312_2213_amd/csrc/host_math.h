// host_math.h -- the host-side FP64 arithmetic of the multicanonical
// iteration: reachable bins, integer acceptance thresholds from the log
// weights, the accumulated-statistics recursion, flatness, and reweighting
// (Eq. 2).  Plain C++ with no HIP dependency, so it can also be built on its
// own (with sanitizers) for checking.
#pragma once

#include <stdint.h>

// Bins of the binned quantity (value lo + b * step) that some lattice
// configuration takes; model is MUCA_ISING, MUCA_POTTS or MUCA_MUMA.
void muca_reachable_mask(int model, int q, int lo, int step, int n_sites, int n_bins, uint8_t *m);

// min(1, exp(D)) as an integer threshold on a uniform 32-bit word r: accept
// iff r < T, with T = 0xffffffff meaning "always".
uint32_t muca_threshold_of(double D);

// T[b * n_cols + j] for every bin b and column j of a lattice model (Ising:
// 5 columns, dE = 4j - 8; Potts: 9 columns, dE_unsat = j - 4; MUMA: 10
// columns, the magnetisation step by (j & 1) and dE = 4 (j >> 1) - 8 at
// inverse temperature beta).  A target bin outside the range gives 0.
void muca_lattice_thresholds(int model, double beta, int n_bins, int n_cols, const double *lnW, uint32_t *T);

// Accumulated-statistics recursion on consecutive bins of the set m; lnW is
// rebuilt as the running sum of lnR (0 at the set's first bin).
void muca_recursion(int B, const uint8_t *m, const uint64_t *H, double *lnR, double *P, double *lnW);

// min / mean of H over the set m (0 if the set is empty or H is zero there).
double muca_flatness(int B, const uint8_t *m, const uint64_t *H);

// Eq. 2 over the bins: out = { <v>/N, beta^2 Var(v)/N, <v>, ln Z } (muma =
// false: canonical at beta from a run with log weights lnW), or { <|v|>/N,
// <v^2>/N^2, <v>/N, ln Z } for a multimagnetic run (beta unused).
void muca_reweight_bins(int B, const uint64_t *H, const double *lnW, const double *val, int nsite, bool muma,
                        double beta, double *out);

// Canonical averages at beta2 from the joint (E, M) histogram h[e * B + b]
// (E = -2N + 4e, M = lo + mstep * b) of a multimagnetic run at beta with log
// weights lnW: out = { <E>/N, beta2^2 Var(E)/N, <|M|>/N, <M^2>/N^2,
// beta2 (<M^2> - <|M|>^2)/N, ln Z }.
void muca_reweight_joint(int NE, int B, const uint64_t *h, const double *lnW, int32_t lo, int32_t mstep, int nsite,
                         double beta, double beta2, double *out);
