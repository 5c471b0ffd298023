// host_math_check.cpp -- runs the host-side arithmetic of host_math.cpp on
// cases read from a text file and prints the results, so that the same
// code the library uses can be built on its own with sanitizers and its
// output compared with an independent implementation.
//
// Input: whitespace-separated tokens, doubles as C hexadecimal floats (%a),
// one case after another:
//   mask <model> <q> <lo> <step> <n_sites> <B>
//   thresholds <model> <beta> <B> <n_cols> lnW[B]
//   recursion <B> mask[B] H[B] lnR[B] P[B]
//   flatness <B> mask[B] H[B]
//   reweight <B> <muma> <nsite> <beta> H[B] lnW[B] val[B]
//   joint <NE> <B> <lo> <mstep> <nsite> <beta> <beta2> h[NE * B] lnW[B]
// Output: one line per case, the results in the same formats.
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_math.h"

namespace {

FILE *in = nullptr;

[[noreturn]] void fail(const char *what)
{
    std::fprintf(stderr, "host_math_check: bad input (%s)\n", what);
    std::exit(2);
}

long long get_int()
{
    long long v;
    if (std::fscanf(in, "%lld", &v) != 1)
        fail("integer");
    return v;
}

double get_double()
{
    char tok[64];
    if (std::fscanf(in, "%63s", tok) != 1)
        fail("double");
    return std::strtod(tok, nullptr);
}

uint64_t get_u64()
{
    unsigned long long v;
    if (std::fscanf(in, "%llu", &v) != 1)
        fail("count");
    return v;
}

template <class T, class F>
std::vector<T> get_n(long long n, F f)
{
    if (n < 0 || n > (1 << 24))
        fail("length");
    std::vector<T> v((size_t)n);
    for (auto &x : v)
        x = (T)f();
    return v;
}

void put_doubles(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        std::printf("%s%a", i ? " " : "", v[i]);
    std::printf("\n");
}

} // namespace

int main(int argc, char **argv)
{
    if (argc != 2)
        fail("usage: host_math_check <cases file>");
    in = std::fopen(argv[1], "r");
    if (!in)
        fail("cannot open the cases file");
    char kind[32];
    while (std::fscanf(in, "%31s", kind) == 1) {
        if (!std::strcmp(kind, "mask")) {
            const int model = (int)get_int(), q = (int)get_int(), lo = (int)get_int(), step = (int)get_int();
            const int n_sites = (int)get_int(), B = (int)get_int();
            std::vector<uint8_t> m((size_t)B);
            muca_reachable_mask(model, q, lo, step, n_sites, B, m.data());
            for (int b = 0; b < B; ++b)
                std::printf("%s%d", b ? " " : "", m[b]);
            std::printf("\n");
        } else if (!std::strcmp(kind, "thresholds")) {
            const int model = (int)get_int();
            const double beta = get_double();
            const int B = (int)get_int(), NC = (int)get_int();
            const auto lnW = get_n<double>(B, get_double);
            std::vector<uint32_t> T((size_t)B * NC);
            muca_lattice_thresholds(model, beta, B, NC, lnW.data(), T.data());
            for (size_t i = 0; i < T.size(); ++i)
                std::printf("%s%" PRIu32, i ? " " : "", T[i]);
            std::printf("\n");
        } else if (!std::strcmp(kind, "recursion")) {
            const int B = (int)get_int();
            const auto m = get_n<uint8_t>(B, get_int);
            const auto H = get_n<uint64_t>(B, get_u64);
            auto lnR = get_n<double>(B, get_double);
            auto P = get_n<double>(B, get_double);
            std::vector<double> lnW((size_t)B);
            muca_recursion(B, m.data(), H.data(), lnR.data(), P.data(), lnW.data());
            std::vector<double> all(lnR);
            all.insert(all.end(), P.begin(), P.end());
            all.insert(all.end(), lnW.begin(), lnW.end());
            put_doubles(all.data(), all.size());
        } else if (!std::strcmp(kind, "flatness")) {
            const int B = (int)get_int();
            const auto m = get_n<uint8_t>(B, get_int);
            const auto H = get_n<uint64_t>(B, get_u64);
            const double f = muca_flatness(B, m.data(), H.data());
            put_doubles(&f, 1);
        } else if (!std::strcmp(kind, "reweight")) {
            const int B = (int)get_int(), muma = (int)get_int(), nsite = (int)get_int();
            const double beta = get_double();
            const auto H = get_n<uint64_t>(B, get_u64);
            const auto lnW = get_n<double>(B, get_double);
            const auto val = get_n<double>(B, get_double);
            double out[4];
            muca_reweight_bins(B, H.data(), lnW.data(), val.data(), nsite, muma != 0, beta, out);
            put_doubles(out, 4);
        } else if (!std::strcmp(kind, "joint")) {
            const int NE = (int)get_int(), B = (int)get_int(), lo = (int)get_int(), mstep = (int)get_int();
            const int nsite = (int)get_int();
            const double beta = get_double(), beta2 = get_double();
            const auto h = get_n<uint64_t>((long long)NE * B, get_u64);
            const auto lnW = get_n<double>(B, get_double);
            double out[6];
            muca_reweight_joint(NE, B, h.data(), lnW.data(), lo, mstep, nsite, beta, beta2, out);
            put_doubles(out, 6);
        } else {
            fail(kind);
        }
    }
    std::fclose(in);
    return 0;
}
