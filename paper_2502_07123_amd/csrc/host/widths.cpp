// Bit-width optimisation of one level (Sections 5 and 6) from the error model's
// sensitivities: the Lagrange widths for a multiplier lambda, lambda by
// golden-section search on the level objective, the greedy integer rounding, and
// the fixed-point kernel's formats of the result.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../../include/mlmc.h"

namespace {

constexpr int NV = MLMC_NVARS;

struct Counts {
    double M[NV];                   // multiplications taking the variable as an operand
    double A[NV];                   // additions taking it as an operand
};

// per sample, on the kernel's operations: fine step mul2 = X s_k, X = X + mul2 (s_k
// from the table); coarse step the whole chain on Zs (which has Z's format)
Counts op_counts(bool mil, int level) {
    Counts c;
    std::memset(&c, 0, sizeof(c));
    const double N = std::ldexp(1.0, level);
    const double Nc = level >= 1 ? N / 2 : 0.0;
    const int s = mil ? MLMC_V_SUM2 : MLMC_V_SUM1;
    for (const double steps : {N, Nc}) {
        c.M[MLMC_V_X] += steps;
        c.M[s] += steps;
        c.A[MLMC_V_X] += steps;
        c.A[MLMC_V_MUL2] += steps;
    }
    c.M[MLMC_V_CON2] += Nc;         // mul1 = con2 zs
    c.M[MLMC_V_Z] += Nc;
    c.A[MLMC_V_CON1] += Nc;         // sum1 = con1c + mul1
    c.A[MLMC_V_MUL1] += Nc;
    if (mil) {
        c.M[MLMC_V_Z] += 2 * Nc;    // zsq = zs zs
        c.A[MLMC_V_ZSQ] += Nc;      // zm1 = zsq - 2
        c.M[MLMC_V_CON3] += Nc;     // mul3 = con3 zm1
        c.M[MLMC_V_ZM1] += Nc;
        c.A[MLMC_V_SUM1] += Nc;     // sum2 = sum1 + mul3
        c.A[MLMC_V_MUL3] += Nc;
    }
    return c;
}

double d_max(int v) { return v == MLMC_V_Z ? 30.0 : 31.0; }

double cost(const Counts& c, const double* d, const int32_t* used) {
    double s = 0.0;
    for (int v = 0; v < NV; ++v)
        if (used[v]) s += 0.5 * c.M[v] * d[v] * d[v] + c.A[v] * d[v];
    return s;
}

// V_indep (eq. optimistic), plus the table's term S_Z MSE when rng
double v_indep(const mlmc_error_model& m, const double* d, bool rng) {
    double s = 0.0;
    for (int v = 0; v < NV; ++v)
        if (m.used[v]) s += m.S[v] * std::pow(4.0, m.e[v] - d[v]);
    s /= 12.0;
    return s + (rng ? m.S[MLMC_V_Z] * m.mse : 0.0);
}

// root in d of ln4 (S/12) 4^(e-d) = lambda (M d + M') on [0, hi], by bisection; a
// variable that costs nothing (M = M' = 0) takes hi
double solve_d(double S, int e, double Mi, double Ai, double lam, double hi) {
    if (Mi == 0.0 && Ai == 0.0) return hi;
    const double ln4 = std::log(4.0);
    auto g = [&](double d) { return ln4 * S / 12.0 * std::pow(4.0, e - d) - lam * (Mi * d + Ai); };
    double lo = 0.0;
    if (g(lo) <= 0.0) return lo;
    if (g(hi) >= 0.0) return hi;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (g(mid) > 0.0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

void widths_for(const mlmc_error_model& m, const Counts& c, double lam, double* d) {
    for (int v = 0; v < NV; ++v)
        d[v] = m.used[v] ? solve_d(m.S[v], m.e[v], c.M[v], c.A[v], lam, d_max(v)) : 0.0;
}

// the level objective sqrt(V_l C(d)) + sqrt(V^D(d) C_l) (Section 6)
double objective(const mlmc_error_model& m, const Counts& c, const double* d, double C_l, bool rng) {
    return std::sqrt(m.V_level * cost(c, d, m.used)) + std::sqrt(v_indep(m, d, rng) * C_l);
}

// lambda at which a uniform width du is stationary: sum dV/dd + lambda sum dC/dd = 0
double uniform_lambda(const mlmc_error_model& m, const Counts& c, double du) {
    double dV = 0.0, dC = 0.0;
    for (int v = 0; v < NV; ++v) {
        if (!m.used[v]) continue;
        dV += m.S[v] * std::pow(4.0, m.e[v] - du);
        dC += c.M[v] * du + c.A[v];
    }
    dV *= -std::log(4.0) / 12.0;
    return -dV / dC;
}

}  // namespace

extern "C" mlmc_status mlmc_optimise_widths(const mlmc_error_model* model, double c_rng, int32_t rng_term,
                                            mlmc_width_plan* out) {
    if (!model || !out) return MLMC_E_INVALID;
    if (model->struct_size != sizeof(mlmc_error_model) || out->struct_size != sizeof(mlmc_width_plan))
        return MLMC_E_VERSION;
    const mlmc_error_model& m = *model;
    if (m.level < 0 || m.level > 20 || (m.scheme != MLMC_EULER && m.scheme != MLMC_MILSTEIN) ||
        !(c_rng > 0.0) || !std::isfinite(c_rng) || !(m.V_level >= 0.0))
        return MLMC_E_INVALID;
    for (int v = 0; v < NV; ++v)
        if (m.used[v] && (!(m.S[v] >= 0.0) || !std::isfinite(m.S[v]) || m.e[v] < -1074 || m.e[v] > 1024))
            return MLMC_E_INVALID;
    const bool mil = m.scheme == MLMC_MILSTEIN;
    const bool rng = rng_term != 0;
    const Counts c = op_counts(mil, m.level);
    const double C_l = std::ldexp(1.0, m.level) * c_rng;

    // bracket: the lambdas of the uniform widths 4..16
    double lo = HUGE_VAL, hi = -HUGE_VAL;
    for (int du = 4; du <= 16; ++du) {
        const double l = std::log(uniform_lambda(m, c, du));
        lo = std::min(lo, l);
        hi = std::max(hi, l);
    }
    if (!std::isfinite(lo) || !std::isfinite(hi)) return MLMC_E_INVALID;
    double d[NV];
    auto obj = [&](double t) {
        widths_for(m, c, std::exp(t), d);
        return objective(m, c, d, C_l, rng);
    };
    // golden-section search (200 reductions) of the unimodal objective in log lambda
    const double g = (std::sqrt(5.0) - 1.0) / 2.0;
    double a = lo, b = hi;
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = obj(x1), f2 = obj(x2);
    for (int it = 0; it < 200; ++it) {
        if (f1 < f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            f1 = obj(x1);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            f2 = obj(x2);
        }
    }
    const double t = 0.5 * (a + b);
    std::memset(reinterpret_cast<uint8_t*>(out) + sizeof(uint32_t), 0, sizeof(*out) - sizeof(uint32_t));
    out->lambda = std::exp(t);
    out->objective = obj(t);
    double dr[NV];
    widths_for(m, c, out->lambda, dr);
    for (int v = 0; v < NV; ++v) out->d_real[v] = dr[v];

    // greedy rounding (eq. ratio_lagr): floor, then one bit at a time in decreasing
    // order of variance gained per cost until V^D(d) <= V^D(d_real)
    double di[NV];
    for (int v = 0; v < NV; ++v) di[v] = std::floor(dr[v]);
    const double target = v_indep(m, dr, rng);
    struct Cand {
        double key;
        int v;
    };
    Cand cand[NV];
    int nc = 0;
    const double v0 = v_indep(m, di, rng), c0 = cost(c, di, m.used);
    for (int v = 0; v < NV; ++v) {
        if (!m.used[v] || di[v] >= d_max(v)) continue;
        double up[NV];
        std::memcpy(up, di, sizeof(up));
        up[v] += 1.0;
        const double dv = v0 - v_indep(m, up, rng);
        const double dc = cost(c, up, m.used) - c0;
        cand[nc++] = Cand{dc > 0.0 ? -(dv / dc) : -HUGE_VAL, v};
    }
    std::stable_sort(cand, cand + nc, [](const Cand& x, const Cand& y) {
        return x.key < y.key || (x.key == y.key && x.v < y.v);
    });
    for (int k = 0; k < nc; ++k) {
        if (v_indep(m, di, rng) <= target) break;
        di[cand[k].v] += 1.0;
    }
    for (int v = 0; v < NV; ++v) out->d_int[v] = static_cast<int32_t>(di[v]);
    out->v_indep = v_indep(m, di, rng);
    out->cost = cost(c, di, m.used);

    // the best uniform width of 4..16 (capped at d_max)
    double best = HUGE_VAL;
    for (int du = 4; du <= 16; ++du) {
        double u[NV];
        for (int v = 0; v < NV; ++v) u[v] = m.used[v] ? std::min<double>(du, d_max(v)) : 0.0;
        const double o = objective(m, c, u, C_l, rng);
        if (o < best) {
            best = o;
            out->best_uniform = du;
        }
    }
    out->objective_uniform = best;

    // kernel formats: w = d + 1, f = d - e, then no fractional bit that cannot change
    // a result: f <= (Z: 30, else 31) - e and >= 0, products f_dst <= f_a + f_b, sums
    // f_dst <= max(f_a, f_b) with |f_a - f_b| <= 30, zsq f <= 30 (three passes)
    int f[NV], e[NV];
    for (int v = 0; v < NV; ++v) {
        e[v] = m.e[v];
        f[v] = out->d_int[v] - e[v];
    }
    auto cap = [&](int v) { f[v] = std::max(std::min(f[v], (v == MLMC_V_Z ? 30 : 31) - e[v]), 0); };
    auto prod = [&](int dst, int a2, int b2) {
        f[dst] = std::min(f[dst], f[a2] + f[b2]);
        cap(dst);
    };
    auto add = [&](int dst, int a2, int b2) {
        const int h = f[a2] >= f[b2] ? a2 : b2, l = f[a2] >= f[b2] ? b2 : a2;
        if (f[h] - f[l] > 30) {
            f[h] = f[l] + 30;
            cap(h);
        }
        f[dst] = std::min(f[dst], std::max(f[a2], f[b2]));
        cap(dst);
    };
    for (int v = 0; v < NV; ++v)
        if (m.used[v]) cap(v);
    for (int pass = 0; pass < 3; ++pass) {
        prod(MLMC_V_MUL1, MLMC_V_CON2, MLMC_V_Z);
        add(MLMC_V_SUM1, MLMC_V_CON1, MLMC_V_MUL1);
        int s = MLMC_V_SUM1;
        if (mil) {
            prod(MLMC_V_ZSQ, MLMC_V_Z, MLMC_V_Z);
            f[MLMC_V_ZSQ] = std::min(f[MLMC_V_ZSQ], 30);
            cap(MLMC_V_ZSQ);
            add(MLMC_V_ZM1, MLMC_V_ZSQ, MLMC_V_ZSQ);
            prod(MLMC_V_MUL3, MLMC_V_CON3, MLMC_V_ZM1);
            add(MLMC_V_SUM2, MLMC_V_SUM1, MLMC_V_MUL3);
            s = MLMC_V_SUM2;
        }
        prod(MLMC_V_MUL2, MLMC_V_X, s);
        add(MLMC_V_X, MLMC_V_X, MLMC_V_MUL2);
    }
    for (int v = 0; v < NV; ++v) {
        out->frac_bits[v] = m.used[v] ? f[v] : 0;
        out->word_bits[v] = m.used[v] ? f[v] + e[v] + 1 : 0;
    }
    return MLMC_OK;
}
