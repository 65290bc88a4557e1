// abi_stats.cpp -- equilibrium averages of a record series (product side):
// means, Flyvbjerg-Petersen blocked errors, the Binder cumulant and its
// jackknife error, specific heat and susceptibility.
#include <cmath>
#include <cstring>
#include <vector>

#include "abi_internal.h"

using namespace mcabi;

namespace {

double mean_of(const std::vector<double> &x)
{
    double s = 0.0;
    for (double v : x) s += v;
    return x.empty() ? 0.0 : s / (double)x.size();
}

// Standard error of the mean of a correlated series: repeated pairwise
// blocking (Flyvbjerg & Petersen 1989), maximum over levels with >= 32 blocks.
double blocked_error(std::vector<double> x)
{
    double best = 0.0;
    while (x.size() >= 32) {
        const double m = mean_of(x);
        double v = 0.0;
        for (double a : x) v += (a - m) * (a - m);
        v /= (double)(x.size() - 1);
        best = std::max(best, std::sqrt(v / (double)x.size()));
        std::vector<double> y(x.size() / 2);
        for (size_t i = 0; i < y.size(); ++i) y[i] = 0.5 * (x[2 * i] + x[2 * i + 1]);
        x.swap(y);
    }
    if (best == 0.0 && x.size() > 1) {
        const double m = mean_of(x);
        double v = 0.0;
        for (double a : x) v += (a - m) * (a - m);
        best = std::sqrt(v / (double)(x.size() - 1) / (double)x.size());
    }
    return best;
}

// Error of the Binder cumulant U4 = 1 - <m^4>/(3 <m^2>^2): delete-one-block
// jackknife over B = min(32, n) contiguous blocks, record i in block
// floor(B i / n).
double binder_jackknife(const std::vector<double> &m2, const std::vector<double> &m4)
{
    const size_t n = m2.size();
    const size_t B = std::min<size_t>(32, n);
    if (B < 2) return 0.0;
    std::vector<double> s2(B, 0.0), s4(B, 0.0), cnt(B, 0.0);
    double t2 = 0.0, t4 = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const size_t b = (size_t)(((unsigned __int128)i * B) / n);
        s2[b] += m2[i];
        s4[b] += m4[i];
        cnt[b] += 1.0;
        t2 += m2[i];
        t4 += m4[i];
    }
    std::vector<double> u(B);
    double mu = 0.0;
    for (size_t b = 0; b < B; ++b) {
        const double rest = (double)n - cnt[b];
        const double q2 = (t2 - s2[b]) / rest, q4 = (t4 - s4[b]) / rest;
        u[b] = 1.0 - q4 / (3.0 * q2 * q2);
        mu += u[b];
    }
    mu /= (double)B;
    double v = 0.0;
    for (double x : u) v += (x - mu) * (x - mu);
    return std::sqrt(v * (double)(B - 1) / (double)B);
}

} // namespace

extern "C" {

mc_status mc_series_stats(const mc_obs *series, uint64_t n, uint64_t stride, double T,
                          mc_stats *out)
{
    if (!series || !out) return fail(MC_E_ARG, "NULL argument");
    if (n < 2 || stride < 1) return fail(MC_E_ARG, "need n >= 2 records and stride >= 1");
    std::vector<double> am(n), m2(n), m4(n), e(n), E(n);
    double acc = 0.0;
    const double N = (double)series[0].n_sites;
    for (uint64_t i = 0; i < n; ++i) {
        const mc_obs &o = series[i * stride];
        const double q = o.M[0] * o.M[0] + o.M[1] * o.M[1] + o.M[2] * o.M[2];
        am[i] = std::sqrt(q);
        m2[i] = q;
        m4[i] = q * q;
        E[i] = o.E;
        e[i] = o.E / N;
        acc += (double)o.n_accepted / N;
    }
    std::memset(out, 0, sizeof *out);
    out->n = n;
    out->abs_m = mean_of(am);
    out->abs_m_err = blocked_error(am);
    out->m2 = mean_of(m2);
    out->m2_err = blocked_error(m2);
    out->m4 = mean_of(m4);
    out->m4_err = blocked_error(m4);
    out->e = mean_of(e);
    out->e_err = blocked_error(e);
    out->U4 = 1.0 - out->m4 / (3.0 * out->m2 * out->m2);
    out->U4_err = binder_jackknife(m2, m4);
    out->acceptance = acc / (double)n;
    if (T > 0.0 && std::isfinite(T)) {
        const double mE = mean_of(E);
        double vE = 0.0;
        for (double v : E) vE += (v - mE) * (v - mE);
        vE /= (double)n;
        out->C = vE / (N * T * T);
        out->chi = N * (out->m2 - out->abs_m * out->abs_m) / T;
    } else {
        out->C = NAN;
        out->chi = NAN;
    }
    return MC_OK;
}

} // extern "C"
