// polymer_host.cpp -- host side of bead-spring polymer runs: workspace,
// initial energies, the B x B threshold matrix and the sweep launches.
//
// Energies follow Eq. 7 of arXiv:1312.2213 in the parametrisation of the
// polymer workload: LJ (eps, sigma) on |i-j| >= 2 cut at r_c and shifted,
// FENE -(K/2) R^2 ln(1 - ((r - r0)/R)^2) on bonds.  The initial total energy
// is summed over pairs i < j in ascending order; bins are
// floor((E - x_lo) * n_bins / (x_hi - x_lo)) on [x_lo, x_hi).
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "muca_internal.h"
#include "runtime_internal.h"

using namespace muca;

static size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

static PolymerConsts consts_of(const muca_config *c)
{
    PolymerConsts k;
    k.lj_eps = c->lj_eps;
    k.lj_sigma = c->lj_sigma;
    k.lj_rcut = c->lj_rcut;
    const double sr2 = (c->lj_sigma * c->lj_sigma) / (c->lj_rcut * c->lj_rcut);
    const double sr6 = sr2 * sr2 * sr2;
    k.lj_shift = 4.0 * c->lj_eps * (sr6 * sr6 - sr6);
    k.fene_pref = 0.5 * c->fene_k * c->fene_R * c->fene_R;
    k.fene_r0 = c->fene_r0;
    k.fene_R = c->fene_R;
    k.x_lo = c->x_lo;
    k.x_hi = c->x_hi;
    k.scale = (double)c->n_bins / (c->x_hi - c->x_lo);
    return k;
}

int muca_polymer_geometry(const muca_config *c, Geometry *g)
{
    if (c->n_beads < 2 || c->n_beads > 128)
        return muca_fail(MUCA_E_ARG, "n_beads %d outside 2..128", c->n_beads);
    if (c->moves != 0 && c->moves != 1)
        return muca_fail(MUCA_E_ARG, "moves %d: 0 (shifts) or 1 (shifts, rotations, double bridging)", c->moves);
    if (c->n_bins < 2 || c->n_bins > 8192 || !(c->x_hi > c->x_lo))
        return muca_fail(MUCA_E_ARG, "bad energy binning (%d bins on [%g, %g))", c->n_bins, c->x_lo, c->x_hi);
    if (!(c->fene_R > 0.0) || !(c->lj_rcut > 0.0) || !(c->lj_sigma > 0.0) || !(c->step > 0.0f))
        return muca_fail(MUCA_E_ARG, "bad potential parameters");
    g->n_sites = c->n_beads;
    g->n_bins = c->n_bins;
    g->n_cols = c->n_bins;
    g->cpb = c->chains_per_block ? c->chains_per_block : 4;
    if (g->cpb < 1 || g->cpb > 4)
        return muca_fail(MUCA_E_ARG, "polymer chains_per_block %d outside 1..4", g->cpb);
    while (g->c_pad % g->cpb)
        g->cpb /= 2;
    // bead slots per chain: lane j of the chain's wavefront holds bead j
    // (and bead j + 64 when n_beads > 64)
    g->lpc = c->n_beads > 64 ? 128 : 64;
    const size_t S = (size_t)g->lpc;
    size_t off = 0;
    g->off_words = off; // positions, float4 per bead slot
    off = align256(off + (size_t)g->c_pad * S * 16);
    g->off_energy = off; // bond energies [c_pad][S] then running energies [c_pad]
    off = align256(off + (size_t)g->c_pad * S * 8 + (size_t)g->c_pad * 8);
    g->off_bins = off;
    off = align256(off + (size_t)g->c_pad * 4);
    g->off_values = off;
    g->off_table = off;
    off = align256(off + (size_t)g->n_bins * g->n_bins * 4);
    g->off_hist = off; // histogram, then the count of accepted moves
    off = align256(off + (size_t)(g->n_bins + 1) * 8);
    g->ws_bytes = off;
    return MUCA_OK;
}

namespace {
double pair_energy(const muca_config *c, const PolymerConsts &k, int i, int j, double r2, bool *broken)
{
    const int sep = i > j ? i - j : j - i;
    if (sep == 1) {
        const double r = std::sqrt(r2);
        const double t = (r - c->fene_r0) / c->fene_R;
        const double arg = 1.0 - t * t;
        if (!(arg > 0.0)) {
            *broken = true;
            return 0.0;
        }
        return -k.fene_pref * std::log(arg);
    }
    if (r2 < c->lj_rcut * c->lj_rcut) {
        const double sr2 = (c->lj_sigma * c->lj_sigma) / r2;
        const double sr6 = sr2 * sr2 * sr2;
        return 4.0 * c->lj_eps * (sr6 * sr6 - sr6) - k.lj_shift;
    }
    return 0.0;
}

double d2(const float *a, const float *b)
{
    const double dx = (double)a[0] - (double)b[0];
    const double dy = (double)a[1] - (double)b[1];
    const double dz = (double)a[2] - (double)b[2];
    return dx * dx + dy * dy + dz * dz;
}

int32_t bin_of(const muca_config *c, const PolymerConsts &k, double E)
{
    if (!(E >= c->x_lo) || !(E < c->x_hi))
        return -1;
    const double f = std::floor((E - c->x_lo) * k.scale);
    if (f < 0.0 || f >= (double)c->n_bins)
        return -1;
    return (int32_t)f;
}
} // namespace

int muca_polymer_init(muca_run *r, const float *h_pos)
{
    const muca_config *c = &r->cfg;
    const Geometry &g = r->g;
    if (!h_pos)
        return muca_fail(MUCA_E_ARG, "polymer runs need initial positions");
    const PolymerConsts k = consts_of(c);
    const int N = c->n_beads, C = c->n_chains;
    const size_t S = (size_t)g.lpc;
    std::vector<float> pos((size_t)g.c_pad * S * 4, 0.0f);
    std::vector<double> bond((size_t)g.c_pad * S + g.c_pad, 0.0);
    std::vector<int32_t> bins(g.c_pad, 0);
    double *energy = bond.data() + (size_t)g.c_pad * S;
    for (int ch = 0; ch < g.c_pad; ++ch) {
        // padding chains copy chain 0: valid states, never histogrammed
        const float *src = h_pos + (size_t)(ch < C ? ch : 0) * N * 3;
        for (int j = 0; j < N; ++j)
            for (int a = 0; a < 3; ++a)
                pos[((size_t)ch * S + j) * 4 + a] = src[3 * j + a];
        bool broken = false;
        double e = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j)
                e += pair_energy(c, k, i, j, d2(src + 3 * i, src + 3 * j), &broken);
        for (int j = 0; j + 1 < N; ++j)
            bond[(size_t)ch * S + j] = pair_energy(c, k, j, j + 1, d2(src + 3 * j, src + 3 * j + 3), &broken);
        energy[ch] = e;
        bins[ch] = broken ? -1 : bin_of(c, k, e);
        if (bins[ch] < 0)
            return muca_fail(MUCA_E_RANGE, "chain %d starts outside [%g, %g) or with a broken bond", ch, c->x_lo,
                             c->x_hi);
    }
    r->d_words = (uint32_t *)(r->ws + g.off_words);
    r->d_energy = (double *)(r->ws + g.off_energy);
    r->d_bins = (int32_t *)(r->ws + g.off_bins);
    r->d_table = (uint32_t *)(r->ws + g.off_table);
    r->d_hist = (unsigned long long *)(r->ws + g.off_hist);
    r->mask.assign(g.n_bins, 0);
    try {
        r->T.assign((size_t)g.n_bins * g.n_bins, 0u);
    } catch (const std::bad_alloc &) {
        return muca_fail(MUCA_E_NOMEM, "polymer init: pinned host memory for the %d x %d threshold table", g.n_bins,
                         g.n_bins);
    }
    hipError_t e = hipMemcpy(r->d_words, pos.data(), pos.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(r->d_energy, bond.data(), bond.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(r->d_bins, bins.data(), bins.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_fill_u64(r->d_hist, g.n_bins + 1, r->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess)
        return muca_fail(MUCA_E_HIP, "polymer init: %s", hipGetErrorString(e));
    muca_polymer_build(r);
    return muca_upload_thresholds(r);
}

// T[b][b'] = threshold of lnW(b') - lnW(b); rows built in parallel threads
// (each entry is the same pure function of two doubles).
void muca_polymer_build(muca_run *r)
{
    const int B = r->g.n_bins;
    const double *lnW = r->lnW.data();
    uint32_t *T = r->T.data();
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt < 1 ? 1 : (nt > 16 ? 16 : nt);
    auto work = [&](unsigned t) {
        for (int b = (int)t; b < B; b += (int)nt)
            for (int bp = 0; bp < B; ++bp)
                T[(size_t)b * B + bp] = muca_threshold_of(lnW[bp] - lnW[b]);
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t)
        th.emplace_back(work, t);
    work(0);
    for (auto &x : th)
        x.join();
}

int muca_polymer_enqueue(muca_run *r, int64_t sweeps, bool record, hipStream_t s)
{
    const Geometry &g = r->g;
    const PolymerConsts k = consts_of(&r->cfg);
    const int64_t max_chunk = (int64_t)(0xFFFFFFFFll / g.cpb) - 1;
    int64_t done = 0;
    while (done < sweeps) {
        const int64_t n = std::min<int64_t>(sweeps - done, std::min<int64_t>(max_chunk, 1 << 30));
        PolymerArgs a{};
        a.pos = (float4 *)r->d_words;
        a.bond = r->d_energy;
        a.energy = r->d_energy + (size_t)g.c_pad * g.lpc;
        a.bins = r->d_bins;
        a.thresholds = r->d_table;
        a.hist = r->d_hist;
        a.k0 = (uint32_t)(r->cfg.seed & 0xffffffffu);
        a.k1 = (uint32_t)(r->cfg.seed >> 32);
        a.g0 = r->sweep;
        a.n_sweeps = (int32_t)n;
        a.n_chains = r->cfg.n_chains;
        a.c_pad = g.c_pad;
        a.n_bins = g.n_bins;
        a.n_beads = r->cfg.n_beads;
        a.record = record ? 1 : 0;
        a.chains_per_block = g.cpb;
        a.chain0 = r->cfg.chain0;
        a.step = r->cfg.step;
        a.moves = r->cfg.moves;
        a.accepts = r->d_hist + g.n_bins;
        hipError_t e = launch_polymer_sweeps(a, k, s);
        if (e != hipSuccess) {
            r->poisoned = true;
            return muca_fail(MUCA_E_HIP, "polymer sweeps: %s", hipGetErrorString(e));
        }
        r->sweep += (uint32_t)n;
        done += n;
    }
    return MUCA_OK;
}

int muca_polymer_state(muca_run *r, int32_t chain0, int32_t count, float *pos, int32_t *bins, double *energy)
{
    const Geometry &g = r->g;
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e == hipSuccess && bins && count)
        e = hipMemcpy(bins, r->d_bins + chain0, (size_t)count * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && energy && count)
        e = hipMemcpy(energy, r->d_energy + (size_t)g.c_pad * g.lpc + chain0, (size_t)count * 8,
                      hipMemcpyDeviceToHost);
    if (e == hipSuccess && pos && count) {
        const size_t S = (size_t)g.lpc;
        std::vector<float> p((size_t)count * S * 4);
        e = hipMemcpy(p.data(), (const float *)r->d_words + (size_t)chain0 * S * 4, p.size() * 4,
                      hipMemcpyDeviceToHost);
        for (int k = 0; k < count && e == hipSuccess; ++k)
            for (int j = 0; j < r->cfg.n_beads; ++j)
                for (int a = 0; a < 3; ++a)
                    pos[((size_t)k * r->cfg.n_beads + j) * 3 + a] = p[((size_t)k * S + j) * 4 + a];
    }
    if (e != hipSuccess) {
        r->poisoned = true;
        return muca_fail(MUCA_E_HIP, "polymer state: %s", hipGetErrorString(e));
    }
    return MUCA_OK;
}
