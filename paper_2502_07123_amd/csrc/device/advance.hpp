// The adaptive nested MLMC driver's decisions for one option (Sections 2.1, 2.2
// and 6) on a plain-data state, compiled for the host and for the device from this
// one source, so that a run driven by the host and a run driven by the device
// kernels make the same decisions from the same sums:
//   * pilot samples on every level up to L (R12);
//   * per-level estimator once a level's pilot has landed (R35): the nested pair
//     (approximate + correction) only while (sqrt(V~ c~) + sqrt(V^D c^D))^2 <= V~ c,
//     else plain samples;
//   * the optimal allocation N = ceil(theta^-1 eps^-2 sqrt(V/C) sum sqrt(V C)) over
//     all (level, estimator) pairs with C = 2^l c_estimator (R10, R11);
//   * the bias test over the last three levels with alpha = 1 (R34), adding level
//     L + 1 while it fails and L < L_max.
// Variances by R9.  Only IEEE operations that are correctly rounded everywhere
// (+ - * /, sqrt, ceil, ldexp, fabs) and no contraction.
#pragma once
#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "../../../include/mlmc.h"

namespace mlmc {

constexpr int RUN_LEVELS = MLMC_MAX_LEVELS;
constexpr int RUN_MAX_PEND = 2 * RUN_LEVELS;

// Sums of one (level, estimator) for the option's payoff.
struct EstSums {
    uint64_t n;
    double s1, s2, e1, e2;
    int64_t i1;
    uint64_t i2lo, i2hi;
    uint64_t sat, nonfinite;
};

struct RunPending {
    int32_t level, est;
    uint64_t n;
};

struct RunState {
    // configuration
    double eps;                 // eps on the normalised price
    double theta;
    double cost[3];             // per fine path-step, by estimator (PLAIN, APPROX, CORR)
    uint64_t n_pilot;
    int32_t nested, L_min, L_max;
    // progress
    int32_t L, done, sweeps;
    uint8_t plain_lv[RUN_LEVELS], decided[RUN_LEVELS];
    uint8_t pad0[6];
    uint64_t path_steps;
    EstSums sums[RUN_LEVELS][3];
    // the works of the next sweep (set by run_advance)
    int32_t n_pend;
    int32_t pad1;
    RunPending pend[RUN_MAX_PEND];
};

__host__ __device__ inline void run_init(RunState& o, double eps_norm, double theta, const double cost[3],
                                         uint64_t n_pilot, int nested, int L_min, int L_max) {
    char* p = reinterpret_cast<char*>(&o);
    for (size_t i = 0; i < sizeof(RunState); ++i) p[i] = 0;
    o.eps = eps_norm;
    o.theta = theta;
    for (int e = 0; e < 3; ++e) o.cost[e] = cost[e];
    o.n_pilot = n_pilot;
    o.nested = nested;
    o.L_min = L_min;
    o.L_max = L_max;
    o.L = L_min;
}

__host__ __device__ inline bool run_level_plain(const RunState& o, int l) { return !o.nested || o.plain_lv[l]; }
__host__ __device__ inline int run_n_est(const RunState& o, int l) { return run_level_plain(o, l) ? 1 : 2; }
__host__ __device__ inline int run_est_at(const RunState& o, int l, int i) {
    return run_level_plain(o, l) ? MLMC_EST_PLAIN : (i == 0 ? MLMC_EST_APPROX : MLMC_EST_CORR);
}

__host__ __device__ inline double est_mean(const EstSums& s) {
#pragma clang fp contract(off)
    return s.n ? s.s1 / static_cast<double>(s.n) : 0.0;
}

__host__ __device__ inline double est_var(const EstSums& s) {
#pragma clang fp contract(off)
    if (s.n < 2) return 0.0;
    const double n = static_cast<double>(s.n);
    const double v = (s.s2 - s.s1 * s.s1 / n) / (n - 1.0);     // R9
    return v < 0.0 ? 0.0 : v;                                   // std::max(v, 0.0)
}

// a += b, field by field (the per-sweep accumulation of a work's sums)
__host__ __device__ inline void est_accumulate(EstSums& a, const EstSums& b) {
#pragma clang fp contract(off)
    a.s1 += b.s1;
    a.s2 += b.s2;
    a.e1 += b.e1;
    a.e2 += b.e2;
    a.i1 += b.i1;
    const uint64_t lo = a.i2lo + b.i2lo;
    a.i2hi += b.i2hi + (lo < a.i2lo ? 1u : 0u);
    a.i2lo = lo;
    a.n += b.n;
    a.sat += b.sat;
    a.nonfinite += b.nonfinite;
}

__host__ __device__ inline void run_push(RunState& o, int level, int est, uint64_t n) {
    if (o.n_pend < RUN_MAX_PEND) {
        o.pend[o.n_pend].level = level;
        o.pend[o.n_pend].est = est;
        o.pend[o.n_pend].n = n;
        o.n_pend += 1;
    }
}

// Remaining bias after level L (R34): max over l = max(1, L-2) .. L of
// |mean_l| 2^(l - L), over 2^1 - 1.
__host__ __device__ inline double run_remaining_bias(const RunState& o) {
#pragma clang fp contract(off)
    const int L = o.L;
    const int lo = L >= 1 ? (L - 2 > 1 ? L - 2 : 1) : 0;
    double r = 0.0;
    for (int l = lo; l <= L; ++l) {
        double m = 0.0;
        for (int i = 0; i < run_n_est(o, l); ++i) m += est_mean(o.sums[l][run_est_at(o, l, i)]);
        const double b = fabs(m) * ldexp(1.0, l - L);
        r = r < b ? b : r;                                      // std::max(r, b)
    }
    return r / (2.0 - 1.0);
}

// The next sweep's works of the option into o.pend (none: the run is done, o.done
// is set).
__host__ __device__ inline void run_advance(RunState& o) {
#pragma clang fp contract(off)
    o.n_pend = 0;
    if (o.done) return;
    for (int l = 0; l <= o.L; ++l)
        for (int i = 0; i < run_n_est(o, l); ++i) {
            const int e = run_est_at(o, l, i);
            const uint64_t have = o.sums[l][e].n;
            if (have < o.n_pilot) run_push(o, l, e, o.n_pilot - have);
        }
    if (o.n_pend) return;
    if (o.nested) {
        for (int l = 0; l <= o.L; ++l) {
            if (o.decided[l]) continue;
            o.decided[l] = 1;
            if (o.plain_lv[l]) continue;
            double Va = est_var(o.sums[l][MLMC_EST_APPROX]);
            double Vc = est_var(o.sums[l][MLMC_EST_CORR]);
            Va = Va < 1e-300 ? 1e-300 : Va;
            Vc = Vc < 1e-300 ? 1e-300 : Vc;
            const double root = sqrt(Va * o.cost[MLMC_EST_APPROX]) + sqrt(Vc * o.cost[MLMC_EST_CORR]);
            if (root * root > Va * o.cost[MLMC_EST_PLAIN]) {
                o.plain_lv[l] = 1;
                EstSums z = {};
                o.sums[l][MLMC_EST_APPROX] = z;
                o.sums[l][MLMC_EST_CORR] = z;
                run_push(o, l, MLMC_EST_PLAIN, o.n_pilot);
            }
        }
        if (o.n_pend) return;
    }
    const double eps = o.eps;
    double lam = 0.0;
    double Vs[RUN_LEVELS][2];                                   // the clamped variances, once
    for (int l = 0; l <= o.L; ++l)
        for (int i = 0; i < run_n_est(o, l); ++i) {
            const int e = run_est_at(o, l, i);
            double V = est_var(o.sums[l][e]);
            V = V < 1e-300 ? 1e-300 : V;
            Vs[l][i] = V;
            lam += sqrt(V * o.cost[e] * ldexp(1.0, l));
        }
    lam /= o.theta * eps * eps;
    for (int l = 0; l <= o.L; ++l)
        for (int i = 0; i < run_n_est(o, l); ++i) {
            const int e = run_est_at(o, l, i);
            const double V = Vs[l][i];
            const double target = ceil(lam * sqrt(V / (o.cost[e] * ldexp(1.0, l))));
            const uint64_t t = target > 1.8e19 ? UINT64_MAX : static_cast<uint64_t>(target);
            if (t > o.sums[l][e].n) run_push(o, l, e, t - o.sums[l][e].n);
        }
    if (o.n_pend) return;
    if (run_remaining_bias(o) > sqrt(1.0 - o.theta) * eps && o.L < o.L_max) {
        o.L += 1;
        // a new level above a plain level l >= 1 starts plain
        if (o.nested && o.L - 1 >= 1 && o.plain_lv[o.L - 1]) {
            o.plain_lv[o.L] = 1;
            o.decided[o.L] = 1;
        }
        for (int i = 0; i < run_n_est(o, o.L); ++i) run_push(o, o.L, run_est_at(o, o.L, i), o.n_pilot);
        return;
    }
    o.done = 1;
}

}  // namespace mlmc
