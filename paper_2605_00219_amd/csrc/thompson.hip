// Thompson-sampling choice among rasterisation-backward variants (Sec. 4.2):
// a latency belief per variant, a random choice that favours the faster ones,
// and a belief update from each measured latency.
//
// Belief: latencies of arm a are Normal(mu_a, 1 / tau_a) with the conjugate
// Normal-Gamma prior (mu0, kappa0, alpha0, beta0) on (mu_a, tau_a); after n
// observations with mean xbar and squared deviations m2 the posterior is
//   kappa_n = kappa0 + n,  mu_n = (kappa0 mu0 + n xbar) / kappa_n,
//   alpha_n = alpha0 + n / 2,
//   beta_n  = beta0 + m2 / 2 + kappa0 n (xbar - mu0)^2 / (2 kappa_n).
// select draws tau ~ Gamma(alpha_n, rate beta_n), then mu ~ Normal(mu_n,
// 1 / (kappa_n tau)) for every arm and returns the arm with the smallest mu.
// Random numbers: the splitmix64 sequence (Steele, Lea and Flood, 2014),
// uniforms from its top 53 bits, normals by Box-Muller, gammas by Marsaglia
// and Tsang (2000).  Host code only.
#include <cmath>

#include "gs_internal.h"

namespace gs {

static uint64_t splitmix64(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform in (0, 1)
static double uniform01(uint64_t* s) { return ((double)(splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static double normal01(uint64_t* s) {
    const double u1 = uniform01(s), u2 = uniform01(s);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// Gamma(shape a >= 1, scale 1)
static double gamma_draw(uint64_t* s, double a) {
    const double d = a - 1.0 / 3.0, c = 1.0 / std::sqrt(9.0 * d);
    for (;;) {
        double x, v;
        do {
            x = normal01(s);
            v = 1.0 + c * x;
        } while (v <= 0.0);
        v = v * v * v;
        const double u = uniform01(s);
        if (u < 1.0 - 0.0331 * x * x * x * x) return d * v;
        if (std::log(u) < 0.5 * x * x + d * (1.0 - v + std::log(v))) return d * v;
    }
}

static void posterior(const gs_ts_state& st, int a, double* mu, double* kappa, double* alpha, double* beta) {
    const double n = st.n[a];
    *kappa = st.kappa0 + n;
    *mu = (st.kappa0 * st.mu0 + n * st.mean[a]) / *kappa;
    *alpha = st.alpha0 + 0.5 * n;
    const double d = st.mean[a] - st.mu0;
    *beta = st.beta0 + 0.5 * st.m2[a] + st.kappa0 * n * d * d / (2.0 * *kappa);
}

static double draw_mean(gs_ts_state* st, int a) {
    double mu, kappa, alpha, beta;
    posterior(*st, a, &mu, &kappa, &alpha, &beta);
    const double tau = gamma_draw(&st->rng, alpha) / beta;
    return mu + normal01(&st->rng) / std::sqrt(kappa * tau);
}

}  // namespace gs

using namespace gs;

#define TS_REQUIRE(cond, ...)          \
    do {                               \
        if (!(cond)) {                 \
            set_error(__VA_ARGS__);    \
            return GS_ERR_INVALID_ARG; \
        }                              \
    } while (0)

extern "C" {

int gs_ts_init(gs_ts_state* st, int n_arms, uint64_t seed, double mu0, double kappa0, double alpha0,
               double beta0) {
    TS_REQUIRE(st, "gs_ts_init: null state");
    TS_REQUIRE(n_arms >= 1 && n_arms <= GS_TS_MAX_ARMS, "gs_ts_init: n_arms %d not in [1, %d]", n_arms,
               GS_TS_MAX_ARMS);
    TS_REQUIRE(std::isfinite(mu0) && kappa0 > 0.0 && alpha0 >= 1.0 && beta0 > 0.0 && std::isfinite(kappa0) &&
                   std::isfinite(alpha0) && std::isfinite(beta0),
               "gs_ts_init: prior needs finite mu0, kappa0 > 0, alpha0 >= 1, beta0 > 0");
    memset(st, 0, sizeof(*st));
    st->n_arms = n_arms;
    st->rng = seed;
    st->mu0 = mu0;
    st->kappa0 = kappa0;
    st->alpha0 = alpha0;
    st->beta0 = beta0;
    return GS_OK;
}

int gs_ts_select(gs_ts_state* st) {
    TS_REQUIRE(st && st->n_arms >= 1 && st->n_arms <= GS_TS_MAX_ARMS, "gs_ts_select: invalid state");
    int best = 0;
    double best_mu = 0.0;
    for (int a = 0; a < st->n_arms; ++a) {
        const double m = draw_mean(st, a);
        if (a == 0 || m < best_mu) {
            best = a;
            best_mu = m;
        }
    }
    return best;
}

int gs_ts_update(gs_ts_state* st, int arm, double latency) {
    TS_REQUIRE(st && st->n_arms >= 1 && st->n_arms <= GS_TS_MAX_ARMS, "gs_ts_update: invalid state");
    TS_REQUIRE(arm >= 0 && arm < st->n_arms, "gs_ts_update: arm %d not in [0, %d)", arm, st->n_arms);
    TS_REQUIRE(std::isfinite(latency), "gs_ts_update: latency is not finite");
    // Welford's running mean and squared deviations
    st->n[arm] += 1.0;
    const double d = latency - st->mean[arm];
    st->mean[arm] += d / st->n[arm];
    st->m2[arm] += d * (latency - st->mean[arm]);
    return GS_OK;
}

int gs_ts_posterior(const gs_ts_state* st, int arm, double* out) {
    TS_REQUIRE(st && out && st->n_arms >= 1 && st->n_arms <= GS_TS_MAX_ARMS, "gs_ts_posterior: invalid state");
    TS_REQUIRE(arm >= 0 && arm < st->n_arms, "gs_ts_posterior: arm %d not in [0, %d)", arm, st->n_arms);
    posterior(*st, arm, &out[0], &out[1], &out[2], &out[3]);
    return GS_OK;
}

double gs_ts_sample(gs_ts_state* st, int arm) {
    if (!st || arm < 0 || arm >= st->n_arms) return NAN;
    return draw_mean(st, arm);
}

}  // extern "C"
