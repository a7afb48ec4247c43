// Growth statistics (host): the layer sizes read as the distribution of the
// distance from the start over the reached states.
#include <cmath>
#include <cstring>

#include "../../include/cayleygrowth.h"
#include "internal.h"

namespace cg {

namespace {

constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kPi = 3.14159265358979323846;

double normal_cdf(double x, double mu, double sigma) {
    return 0.5 * std::erfc(-(x - mu) / (sigma * std::sqrt(2.0)));
}

// Gumbel of the maximum: F(x) = exp(-exp(-(x - mu) / beta)); of the
// minimum: F(x) = 1 - exp(-exp((x - mu) / beta)).
double gumbel_cdf(double x, double mu, double beta, bool minimum) {
    const double z = (x - mu) / beta;
    return minimum ? -std::expm1(-std::exp(z)) : std::exp(-std::exp(-z));
}

template <class Cdf>
double total_variation(const uint64_t *sizes, int layers, double total, Cdf cdf) {
    // sum over d of |p(d) - mass of [d - 1/2, d + 1/2)|, plus the model's
    // mass outside [-1/2, layers - 1/2)
    double tv = cdf(-0.5) + (1.0 - cdf(layers - 0.5));
    for (int d = 0; d < layers; ++d) {
        const double q = cdf(d + 0.5) - cdf(d - 0.5);
        tv += std::fabs((double)sizes[d] / total - q);
    }
    return 0.5 * tv;
}

}  // namespace

void growth_stats(const uint64_t *sizes, int num_layers, cg_growth_stats_t *o) {
    std::memset(o, 0, sizeof *o);
    int layers = num_layers;
    while (layers > 0 && sizes[layers - 1] == 0) --layers;
    if (layers == 0) throw Error(CG_E_INVAL, "growth has no reached state");
    uint64_t total = 0;
    int mode = 0;
    for (int d = 0; d < layers; ++d) {
        total += sizes[d];
        if (sizes[d] > sizes[mode]) mode = d;
    }
    const double T = (double)total;
    double mean = 0;
    for (int d = 0; d < layers; ++d) mean += (double)d * (double)sizes[d];
    mean /= T;
    double m2 = 0, m3 = 0, m4 = 0;
    for (int d = 0; d < layers; ++d) {
        const double p = (double)sizes[d] / T, x = (double)d - mean;
        m2 += p * x * x;
        m3 += p * x * x * x;
        m4 += p * x * x * x * x;
    }
    o->total = total;
    o->diameter = layers - 1;
    o->mode = mode;
    o->max_layer = sizes[mode];
    o->antipodes = sizes[layers - 1];
    o->mean = mean;
    o->variance = m2;
    o->skewness = m2 > 0 ? m3 / std::pow(m2, 1.5) : 0.0;
    o->kurtosis = m2 > 0 ? m4 / (m2 * m2) - 3.0 : 0.0;
    const double sd = std::sqrt(m2);
    o->gauss_mu = mean;
    o->gauss_sigma = sd;
    o->gumbel_min = o->skewness < 0 ? 1 : 0;
    o->gumbel_beta = sd * std::sqrt(6.0) / kPi;
    o->gumbel_mu = o->gumbel_min ? mean + kEulerGamma * o->gumbel_beta : mean - kEulerGamma * o->gumbel_beta;
    if (sd > 0) {
        o->gauss_tv = total_variation(sizes, layers, T, [&](double x) { return normal_cdf(x, mean, sd); });
        const bool mn = o->gumbel_min != 0;
        o->gumbel_tv = total_variation(sizes, layers, T,
                                       [&](double x) { return gumbel_cdf(x, o->gumbel_mu, o->gumbel_beta, mn); });
    } else {
        o->gauss_tv = o->gumbel_tv = 1.0;  // a point mass: no continuous shape
    }
    o->best_fit = o->gumbel_tv < o->gauss_tv ? 1 : 0;
}

}  // namespace cg
