// Per-level choice of the low-precision side (Section 6's level objective) with a
// gfx950 instruction-class cost model in place of the FPGA bit-operation costs of
// Section 5.
//
// For a level l with error model m (mlmc_error_model) each candidate side
// (arithmetic, q, packing) gets
//   V~   = V_level (the approximate paths' level variance, taken equal to the exact
//          paths'),
//   V^D  = V_round + S_Z MSE_q: the rounding term of the linear model with d = the
//          side's significand bits for every variable (FP32 24, FP16 11: a float's
//          rounding error is at most half an ulp, 2^(e - d - 1) for |x| < 2^e) or the
//          fixed-point widths, plus the Method-1 table's term (reading R16),
//   C~, C^D = 2^l times the cost per fine path-step of the approximate and correction
//          estimators: per instruction class, instructions per path-step over the
//          measured issue rate (wave-instructions per CU per clock),
// and the level objective sqrt(V~ C~) + sqrt(V^D C^D) is minimised over the
// candidates.  Host only.
#include <cmath>
#include <cstring>

#include "../../../include/mlmc.h"
#include "prepare.hpp"

namespace mlmc {
namespace {

constexpr int NV = MLMC_NVARS;

// instruction counts per fine path-step by class
struct ClassCounts {
    double flt = 0, i32 = 0, mad = 0, f64fma = 0, f64add = 0, lds64 = 0, lds32 = 0;
};

double cycles(const ClassCounts& c, const mlmc_gpu_rates& r) {
    return c.flt / r.f32 + c.i32 / r.i32 + c.mad / r.u64_mad + c.f64fma / r.f64_fma + c.f64add / r.f64_add +
           c.lds64 / r.lds_b64 + c.lds32 / r.lds_b32;
}

// The table side's step (FP32 / FP16: Algorithm 1 per operation; FIXED: each
// operation a 32x32 product or an aligned add, then rounding, shift and saturation).
void table_side(ClassCounts& c, int arith, bool mil, int level) {
    const double coarse = level >= 1 ? 0.5 : 0.0;          // one coarse step per fine pair
    if (arith == MLMC_ARITH_FIXED) {
        c.mad += 1.0;                                       // fine: mul2 = X s_k
        c.i32 += 8.0 + 9.0;                                 //       rounding/saturation, X + mul2
        c.mad += coarse * (mil ? 4.0 : 2.0);
        c.i32 += coarse * (mil ? 69.0 : 35.0);
        c.lds64 += 1.0;
    } else {
        c.flt += 2.0 + coarse * (mil ? 9.0 : 5.0);
        (arith == MLMC_ARITH_FP16 ? c.lds32 : c.lds64) += 1.0;
    }
}

// one 32-bit uniform word: a quarter of a Philox4x32-10 call
void philox_word(ClassCounts& c, double share) {
    c.mad += 5.0 * share;
    c.i32 += 7.5 * share;
}

double approx_cost(int arith, int fields, bool mil, int level, const mlmc_gpu_rates& r) {
    ClassCounts c;
    philox_word(c, 1.0 / fields);
    c.i32 += fields > 1 ? 2.0 : 1.0;                        // index (shift; field extract)
    table_side(c, arith, mil, level);
    c.f64add += 4.0 / std::ldexp(1.0, level);               // payoff difference and two sums
    return cycles(c, r);
}

double corr_cost(int arith, bool mil, int level, const mlmc_gpu_rates& r) {
    ClassCounts c;
    philox_word(c, 1.0);
    c.i32 += 1.0;
    c.f64fma += 55.0;                                       // FP64 inverse normal
    c.f64add += 5.0;
    c.f64fma += (mil ? 5.0 : 2.0) + (level >= 1 ? 0.5 * (mil ? 9.0 : 5.0) : 0.0);
    table_side(c, arith, mil, level);
    c.f64add += 8.0 / std::ldexp(1.0, level);
    return cycles(c, r);
}

// V_indep of the linear model with widths d (Section 4.2, eq. optimistic)
double v_round(const mlmc_error_model& m, const double* d) {
    double v = 0.0;
    for (int i = 0; i < NV; ++i)
        if (m.used[i]) v += m.S[i] * std::pow(4.0, m.e[i] - d[i]);
    return v / 12.0;
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" mlmc_status mlmc_gpu_rates_default(mlmc_gpu_rates* out) {
    if (!out) return MLMC_E_INVALID;
    if (out->struct_size != sizeof(mlmc_gpu_rates)) return MLMC_E_VERSION;
    // issue-rate probe on one MI355X (wave-instructions per CU per clock)
    out->f32 = 1.447;
    out->i32 = 1.470;
    out->f64_fma = 0.794;
    out->f64_add = 0.871;
    out->u64_mad = 0.831;
    out->lds_b64 = 0.250;
    out->lds_b32 = 0.500;
    return MLMC_OK;
}

extern "C" mlmc_status mlmc_side_costs(int32_t arith, int32_t table_bits, int32_t packed, int32_t scheme,
                                       int32_t level, const mlmc_gpu_rates* rates, double* c_approx,
                                       double* c_corr) {
    if (!rates || !c_approx || !c_corr) return MLMC_E_INVALID;
    if (rates->struct_size != sizeof(mlmc_gpu_rates)) return MLMC_E_VERSION;
    if (arith != MLMC_ARITH_FP32 && arith != MLMC_ARITH_FP16 && arith != MLMC_ARITH_FIXED) return MLMC_E_INVALID;
    if (table_bits < 1 || table_bits > 12 || level < 0 || level > 20) return MLMC_E_INVALID;
    const double* rr = &rates->f32;
    for (int i = 0; i < 7; ++i)
        if (!(rr[i] > 0.0) || !std::isfinite(rr[i])) return MLMC_E_INVALID;
    const int F = packed ? 32 / table_bits : 1;
    const bool mil = scheme == MLMC_MILSTEIN;
    *c_approx = approx_cost(arith, F, mil, level, *rates);
    *c_corr = corr_cost(arith, mil, level, *rates);
    return MLMC_OK;
}

extern "C" mlmc_status mlmc_choose_precision(const mlmc_error_model* model, const mlmc_gpu_rates* rates,
                                             const mlmc_precision* fixed_formats, mlmc_precision* out,
                                             mlmc_level_choice* info) {
    if (!model || !rates || !out) return MLMC_E_INVALID;
    if (model->struct_size != sizeof(mlmc_error_model) || rates->struct_size != sizeof(mlmc_gpu_rates) ||
        out->struct_size != sizeof(mlmc_precision) || (info && info->struct_size != sizeof(mlmc_level_choice)) ||
        (fixed_formats && fixed_formats->struct_size != sizeof(mlmc_precision)))
        return MLMC_E_VERSION;
    const mlmc_error_model& m = *model;
    if (m.level < 0 || m.level > 20 || (m.scheme != MLMC_EULER && m.scheme != MLMC_MILSTEIN) ||
        !(m.V_level >= 0.0) || !std::isfinite(m.V_level))
        return MLMC_E_INVALID;
    for (int v = 0; v < NV; ++v)
        if (m.used[v] && (!(m.S[v] >= 0.0) || !std::isfinite(m.S[v]) || m.e[v] < -1074 || m.e[v] > 1024))
            return MLMC_E_INVALID;
    const bool mil = m.scheme == MLMC_MILSTEIN;
    const double two_l = std::ldexp(1.0, m.level);

    // candidates: (arith, q, packed) in a fixed order; the first minimum wins
    struct Cand {
        int arith, q, packed;
    };
    static const Cand kCands[] = {
        {MLMC_ARITH_FP32, 8, 1}, {MLMC_ARITH_FP32, 6, 1}, {MLMC_ARITH_FP32, 4, 1},  {MLMC_ARITH_FP32, 10, 0},
        {MLMC_ARITH_FP32, 12, 0}, {MLMC_ARITH_FP16, 8, 1}, {MLMC_ARITH_FP16, 7, 1}, {MLMC_ARITH_FP16, 10, 0},
        {MLMC_ARITH_FIXED, 8, 0}, {MLMC_ARITH_FIXED, 10, 0}, {MLMC_ARITH_FIXED, 12, 0},
    };
    double best = HUGE_VAL, ref = HUGE_VAL;
    int bi = -1;
    double bva = 0, bvc = 0, bca = 0, bcc = 0;
    for (size_t ci = 0; ci < sizeof(kCands) / sizeof(kCands[0]); ++ci) {
        const Cand& c = kCands[ci];
        double d[NV];
        if (c.arith == MLMC_ARITH_FIXED) {
            if (!fixed_formats) continue;
            // widths d = w - 1 of the given formats
            for (int v = 0; v < NV; ++v) d[v] = fixed_formats->word_bits[v] - 1;
        } else {
            const double p = c.arith == MLMC_ARITH_FP32 ? 24.0 : 11.0;
            for (int v = 0; v < NV; ++v) d[v] = p;
        }
        const double vD = v_round(m, d) + m.S[MLMC_V_Z] * table_mse(c.q);
        const double vA = m.V_level;
        const double cA = two_l * approx_cost(c.arith, c.packed ? 32 / c.q : 1, mil, m.level, *rates);
        const double cC = two_l * corr_cost(c.arith, mil, m.level, *rates);
        const double obj = std::sqrt(vA * cA) + std::sqrt(vD * cC);
        if (ci == 0) ref = obj;
        if (obj < best) {
            best = obj;
            bi = static_cast<int>(ci);
            bva = vA;
            bvc = vD;
            bca = cA;
            bcc = cC;
        }
    }
    const Cand& c = kCands[bi];
    const uint32_t sz = out->struct_size;
    if (c.arith == MLMC_ARITH_FIXED) {
        *out = *fixed_formats;
    } else {
        std::memset(out, 0, sizeof(*out));
    }
    out->struct_size = sz;
    out->arith = c.arith;
    out->table_bits = c.q;
    out->packed = c.packed;
    out->rng_method = 1;
    out->exact_side = 0;
    if (info) {
        info->level = m.level;
        info->arith = c.arith;
        info->table_bits = c.q;
        info->packed = c.packed;
        info->v_approx = bva;
        info->v_corr = bvc;
        info->c_approx = bca;
        info->c_corr = bcc;
        info->objective = best;
        info->objective_fp32_q8 = ref;
    }
    return MLMC_OK;
}
