// Host preparation of a level launch: validation, constants, Method-1 table
// (Section 3.1), step tables and kernel-variant choice.
#include "prepare.hpp"

#include <cfloat>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>

#include "../device/fixed.hpp"
#include "../device/norminv.hpp"
#include "../device/paths.hpp"

namespace mlmc {

int popcount32(uint32_t v) {
    int c = 0;
    for (; v; v &= v - 1) ++c;
    return c;
}

static int ctz32(uint32_t v) {
    int c = 0;
    while (v && !(v & 1u)) { v >>= 1; ++c; }
    return c;
}

// ------------------------------------------------------------ Method-1 table
// Phi^-1(k 2^-q) in long double: a bisection-safe start from the FP64 rational
// approximation of the library, then Newton steps on Phi(x) - p with
// Phi(x) = erfc(-x / sqrt 2) / 2 (relative accuracy ~1e-19 in the tails).
static long double Phi_ld(long double x) { return 0.5L * erfcl(-x / sqrtl(2.0L)); }

static long double phi_ld(long double x) {
    return expl(-0.5L * x * x) / sqrtl(2.0L * 3.141592653589793238462643383279502884L);
}

static long double quantile_ld(uint64_t k, int q) {
    const uint64_t n = uint64_t(1) << q;
    if (2 * k == n) return 0.0L;
    const bool upper = 2 * k > n;
    const uint64_t kk = upper ? n - k : k;            // p = kk 2^-q <= 1/2, exact
    const long double p = ldexpl(static_cast<long double>(kk), -q);
    // start: the library's FP64 inverse normal at the nearest 32-bit grid point
    const uint64_t J = static_cast<uint64_t>(ldexpl(p, 32));
    long double x = norminv_f64(static_cast<uint32_t>(J > 0 ? J - 1 : 0));
    for (int it = 0; it < 4; ++it) x -= (Phi_ld(x) - p) / phi_ld(x);
    return upper ? -x : x;
}

// one lock for the table caches (Method 1 and Methods 2/3)
static std::mutex g_tables_mtx;
static const std::vector<long double>& method1_table_nolock(int q);

const std::vector<long double>& method1_table(int q) {
    std::lock_guard<std::mutex> lock(g_tables_mtx);
    return method1_table_nolock(q);
}

// callers hold g_tables_mtx
static const std::vector<long double>& method1_table_nolock(int q) {
    static std::map<int, std::vector<long double>> cache;
    auto it = cache.find(q);
    if (it != cache.end()) return it->second;
    const uint64_t n = uint64_t(1) << q;
    std::vector<long double> a(n + 1);
    for (uint64_t k = 1; k < n; ++k) a[k] = quantile_ld(k, q);
    std::vector<long double> T(n);
    const long double scale = static_cast<long double>(n);
    // T[k] = 2^q (phi(a_k) - phi(a_{k+1})); for interior k written as
    // -phi(a_k) expm1(-(a_{k+1} - a_k)(a_{k+1} + a_k) / 2) to avoid cancellation.
    for (uint64_t k = 0; k < n / 2; ++k) {
        long double v;
        if (k == 0) {
            v = -phi_ld(a[1]);
        } else {
            const long double lo = a[k], hi = a[k + 1];
            v = -phi_ld(lo) * expm1l(-0.5L * (hi - lo) * (hi + lo));
        }
        T[k] = scale * v;
        T[n - 1 - k] = -T[k];                           // antisymmetry
    }
    return cache.emplace(q, std::move(T)).first->second;
}

// ------------------------------------------------ Methods 2 and 3 (Section 3)
// Method 2 (n = 2): j = (chunk 0, chunk 1) of m = q/2 bits each; a chunk with top
// bit s and other bits r contributes +X[r] (s = 1) or -X[M-1-r] (s = 0), M = 2^(m-1)
// (the sign-bit form of Method 1); Z~_j is the sum of the two contributions.  X
// starts as the upper half of the m-bit Method-1 table over sqrt(2); then the Z~
// are ranked (pi(j), ties by j) and X is refitted by least squares against the
// q-bit Method-1 values at pi(j), until pi repeats.  The exact side's uniform takes
// pi(j) as its top q bits.
// Method 3: j = (s, r), r's dyadic interval i = max(1, bit length of r) (intervals
// {0,1}, [2,3], [4,7], ...: q - 1 pairs); on the lower half Z = a_i + b_i r fitted
// by least squares to the Method-1 values, the upper half by antisymmetry.
// Values are formed in FP64 (inputs: the Method-1 values rounded to FP64; fits in
// long double), the precision in which the table builder then rounds them.
namespace {
void m2_chunks(uint32_t j, int q, int m, uint32_t M, uint32_t col[2], double sgn[2]) {
    for (int c = 0; c < 2; ++c) {
        const uint32_t chunk = (j >> (q - m * (c + 1))) & ((1u << m) - 1u);
        const uint32_t s = chunk >> (m - 1), r = chunk & (M - 1u);
        col[c] = s ? r : M - 1u - r;
        sgn[c] = s ? 1.0 : -1.0;
    }
}
// values of the two chunks added in ascending order of value
double m2_value(const std::vector<double>& X, const uint32_t col[2], const double sgn[2]) {
    double a = sgn[0] * X[col[0]], b = sgn[1] * X[col[1]];
    if (b < a) std::swap(a, b);
    return a + b;
}
std::vector<uint32_t> ranks_of(const std::vector<double>& v) {
    std::vector<uint32_t> order(v.size());
    for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return v[a] < v[b]; });
    std::vector<uint32_t> r(v.size());
    for (uint32_t i = 0; i < order.size(); ++i) r[order[i]] = i;
    return r;
}
// least squares by the normal equations, Gaussian elimination with partial pivoting
std::vector<long double> solve_spd(std::vector<long double> A, std::vector<long double> b, size_t M) {
    for (size_t c = 0; c < M; ++c) {
        size_t piv = c;
        for (size_t r = c + 1; r < M; ++r)
            if (fabsl(A[r * M + c]) > fabsl(A[piv * M + c])) piv = r;
        if (piv != c) {
            for (size_t k = 0; k < M; ++k) std::swap(A[c * M + k], A[piv * M + k]);
            std::swap(b[c], b[piv]);
        }
        for (size_t r = c + 1; r < M; ++r) {
            const long double f = A[r * M + c] / A[c * M + c];
            for (size_t k = c; k < M; ++k) A[r * M + k] -= f * A[c * M + k];
            b[r] -= f * b[c];
        }
    }
    std::vector<long double> x(M);
    for (size_t c = M; c-- > 0;) {
        long double t = b[c];
        for (size_t k = c + 1; k < M; ++k) t -= A[c * M + k] * x[k];
        x[c] = t / A[c * M + c];
    }
    return x;
}
}  // namespace

const MethodTable& method_table(int q, int method) {
    static std::map<std::pair<int, int>, MethodTable> cache;
    std::lock_guard<std::mutex> lock(g_tables_mtx);
    auto it = cache.find({q, method});
    if (it != cache.end()) return it->second;
    const uint32_t n = 1u << q;
    std::vector<double> T(n);
    const auto& Tld = method1_table_nolock(q);
    for (uint32_t k = 0; k < n; ++k) T[k] = static_cast<double>(Tld[k]);
    MethodTable out;
    out.z.assign(n, 0.0);
    if (method == 2) {
        const int m = q / 2;
        const uint32_t M = 1u << (m - 1);
        const auto& Hm = method1_table_nolock(m);
        std::vector<double> X(M);
        for (uint32_t r = 0; r < M; ++r) X[r] = static_cast<double>(Hm[M + r]) / std::sqrt(2.0);
        std::vector<uint32_t> pi;
        for (int iter = 0;; ++iter) {
            for (uint32_t j = 0; j < n; ++j) {
                uint32_t col[2];
                double sg[2];
                m2_chunks(j, q, m, M, col, sg);
                out.z[j] = m2_value(X, col, sg);
            }
            std::vector<uint32_t> r = ranks_of(out.z);
            if (r == pi || iter > 5000) {
                out.iterations = iter;                   // least-squares solves made
                break;
            }
            pi = std::move(r);
            std::vector<long double> AtA(size_t(M) * M, 0.0L), Atb(M, 0.0L);
            for (uint32_t j = 0; j < n; ++j) {
                uint32_t col[2];
                double sg[2];
                m2_chunks(j, q, m, M, col, sg);
                const long double t = T[pi[j]];
                for (int a = 0; a < 2; ++a) {
                    Atb[col[a]] += sg[a] * t;
                    for (int b = 0; b < 2; ++b) AtA[size_t(col[a]) * M + col[b]] += sg[a] * sg[b];
                }
            }
            const std::vector<long double> x = solve_spd(AtA, Atb, M);
            for (uint32_t k = 0; k < M; ++k) X[k] = static_cast<double>(x[k]);
        }
        out.perm.resize(n);
        for (uint32_t j = 0; j < n; ++j) out.perm[j] = static_cast<uint16_t>(pi[j]);
    } else {
        const uint32_t half = n / 2;
        std::vector<double> a(q, 0.0), b(q, 0.0);
        auto interval = [](uint32_t r) {
            int bl = 0;
            while (r >> bl) ++bl;
            return bl < 1 ? 1 : bl;
        };
        for (int i = 1; i < q; ++i) {
            const uint32_t lo = i == 1 ? 0u : (1u << (i - 1)), hi = (1u << i) - 1u;
            long double sr = 0, sz = 0;
            const long double cnt = static_cast<long double>(hi - lo + 1);
            for (uint32_t r = lo; r <= hi; ++r) { sr += r; sz += T[r]; }
            const long double rm = sr / cnt, zm = sz / cnt;
            long double sxy = 0, sxx = 0;
            for (uint32_t r = lo; r <= hi; ++r) {
                sxy += (r - rm) * (T[r] - zm);
                sxx += (r - rm) * (r - rm);
            }
            const long double bb = sxy / sxx;
            a[i] = static_cast<double>(zm - bb * rm);
            b[i] = static_cast<double>(bb);
        }
        for (uint32_t j = 0; j < n; ++j) {
            const bool up = j >= half;
            const uint32_t rr = up ? n - 1u - j : j;
            const int i = interval(rr);
            const double prod = b[i] * static_cast<double>(rr);
            const double low = a[i] + prod;
            out.z[j] = up ? -low : low;
        }
    }
    return cache.emplace(std::make_pair(q, method), std::move(out)).first->second;
}

static uint16_t to_half_bits(long double x) {
    // round-to-nearest-even to IEEE binary16 (normal and subnormal; no overflow here)
    const uint16_t sign = std::signbit(x) ? 0x8000u : 0u;
    x = fabsl(x);
    if (x == 0.0L) return sign;
    int e;
    frexpl(x, &e);                                     // x = m 2^e, m in [0.5, 1)
    int exp16 = e - 1;                                 // x = 1.f 2^exp16
    if (exp16 < -14) exp16 = -14;                      // subnormal spacing 2^-24
    const long double m = nearbyintl(ldexpl(x, 10 - exp16));   // 11-bit significand
    long double mm = m;
    int ee = exp16;
    if (mm >= 2048.0L) { mm /= 2.0L; ++ee; }
    const uint32_t mant = static_cast<uint32_t>(mm);
    if (mant < 1024u) return static_cast<uint16_t>(sign | mant);   // subnormal
    return static_cast<uint16_t>(sign | ((ee + 15) << 10) | (mant - 1024u));
}

// x rounded once to binary16 (from the exact value of x)
static _Float16 half_of(long double x) {
    const uint16_t b = to_half_bits(x);
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return h;
}

static bool quantize_ld(long double x, int f, int w, int64_t& out) {
    const long double y = floorl(ldexpl(x, f) + 0.5L);          // R7: ties toward +inf
    const long double hi = ldexpl(1.0L, w - 1) - 1.0L, lo = -ldexpl(1.0L, w - 1);
    if (y > hi || y < lo) return false;
    out = static_cast<int64_t>(y);
    return true;
}

// quantise an FP64 value exactly (saturating silently: constants are inputs)
static int64_t quantize_double(double x, int f, int w) {
    const long double y = floorl(ldexpl(static_cast<long double>(x), f) + 0.5L);
    const long double hi = ldexpl(1.0L, w - 1) - 1.0L, lo = -ldexpl(1.0L, w - 1);
    return static_cast<int64_t>(y > hi ? hi : (y < lo ? lo : y));
}

mlmc_status build_table_bytes(int q, int arith, int frac_bits, void* out, std::string& err) {
    if (q < 1 || q > 16) { err = "table_bits must be 1..16"; return MLMC_E_INVALID; }
    if (!out) { err = "out is NULL"; return MLMC_E_INVALID; }
    const auto& T = method1_table(q);
    const size_t n = T.size();
    switch (arith) {
        case MLMC_ARITH_FP64: {
            double* o = static_cast<double*>(out);
            for (size_t k = 0; k < n; ++k) o[k] = static_cast<double>(T[k]);
            return MLMC_OK;
        }
        case MLMC_ARITH_FP32: {
            float* o = static_cast<float*>(out);
            for (size_t k = 0; k < n; ++k) o[k] = static_cast<float>(T[k]);
            return MLMC_OK;
        }
        case MLMC_ARITH_FP16: {
            uint16_t* o = static_cast<uint16_t*>(out);
            for (size_t k = 0; k < n; ++k) o[k] = to_half_bits(T[k]);
            return MLMC_OK;
        }
        case MLMC_ARITH_FIXED: {
            if (frac_bits < 0 || frac_bits > 28) { err = "frac_bits must be 0..28"; return MLMC_E_INVALID; }
            int32_t* o = static_cast<int32_t*>(out);
            for (size_t k = 0; k < n; ++k) {
                int64_t v;
                if (!quantize_ld(T[k], frac_bits, 32, v)) { err = "table value exceeds 32 bits"; return MLMC_E_INVALID; }
                o[k] = static_cast<int32_t>(v);
            }
            return MLMC_OK;
        }
        default:
            err = "unknown arith";
            return MLMC_E_INVALID;
    }
}

// ---------------------------------------------------------------- validation
static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

mlmc_status validate_problem(const mlmc_problem* p, std::string& err) {
    if (!p) { err = "problem is NULL"; return MLMC_E_INVALID; }
    if (p->struct_size != sizeof(mlmc_problem)) { err = "mlmc_problem.struct_size mismatch"; return MLMC_E_VERSION; }
    if (p->scheme != MLMC_EULER && p->scheme != MLMC_MILSTEIN) { err = "scheme must be EULER or MILSTEIN"; return MLMC_E_INVALID; }
    if (p->payoff_mask == 0 || p->payoff_mask >= (1u << MLMC_NPAYOFF)) { err = "payoff_mask must be a non-empty set of MLMC_PAY_* bits"; return MLMC_E_INVALID; }
    if (!finite_pos(p->S0) || !finite_pos(p->K) || !finite_pos(p->sigma) || !finite_pos(p->T)) { err = "S0, K, sigma and T must be finite and > 0"; return MLMC_E_INVALID; }
    if (!std::isfinite(p->r) || p->r < 0.0) { err = "r must be finite and >= 0"; return MLMC_E_INVALID; }
    if ((p->payoff_mask >> MLMC_PAY_BARRIER) & 1u) {
        if (!std::isfinite(p->barrier) || p->barrier < 0.0 || p->barrier >= p->S0) { err = "barrier must satisfy 0 <= barrier < S0"; return MLMC_E_INVALID; }
    }
    return MLMC_OK;
}

static bool fixed_vars_used(int v, bool mil) {
    switch (v) {
        case MLMC_V_CON3: case MLMC_V_ZSQ: case MLMC_V_ZM1: case MLMC_V_MUL3: case MLMC_V_SUM2:
            return mil;
        default:
            return true;
    }
}

mlmc_status validate_precision(const mlmc_precision* prec, int estimator, const mlmc_problem* p,
                               std::string& err) {
    if (!prec) { err = "precision is NULL"; return MLMC_E_INVALID; }
    if (prec->struct_size != sizeof(mlmc_precision)) { err = "mlmc_precision.struct_size mismatch"; return MLMC_E_VERSION; }
    if (prec->exact_side != 0 && prec->exact_side != 1) { err = "exact_side must be 0 (FP64) or 1 (FP32)"; return MLMC_E_INVALID; }
    if (estimator == MLMC_EST_CORR && prec->exact_side == 1 && prec->arith != MLMC_ARITH_FP32 &&
        prec->arith != MLMC_ARITH_FP16) {
        err = "an FP32 exact side needs an FP32 or FP16 table side";
        return MLMC_E_INVALID;
    }
    if (estimator == MLMC_EST_PLAIN) {
        if (prec->arith != MLMC_ARITH_FP64 && prec->arith != MLMC_ARITH_FP32) { err = "PLAIN supports FP64 and FP32"; return MLMC_E_INVALID; }
        if (prec->packed) { err = "packed indices apply to APPROX only"; return MLMC_E_INVALID; }
        if (prec->rng_method > 1) { err = "PLAIN uses exact normals: rng_method must be 0 or 1"; return MLMC_E_INVALID; }
        return MLMC_OK;
    }
    if (prec->arith != MLMC_ARITH_FP32 && prec->arith != MLMC_ARITH_FP16 && prec->arith != MLMC_ARITH_FIXED) { err = "APPROX/CORR support FP32, FP16 and FIXED arithmetic"; return MLMC_E_INVALID; }
    if (prec->table_bits < 1 || prec->table_bits > 12) { err = "table_bits must be 1..12"; return MLMC_E_INVALID; }
    if (prec->rng_method < 0 || prec->rng_method > 3) { err = "rng_method must be 0..3"; return MLMC_E_INVALID; }
    if (prec->rng_method == 2 && (prec->table_bits % 2 || prec->table_bits < 2)) { err = "Method 2 needs an even table_bits >= 2"; return MLMC_E_INVALID; }
    if (prec->rng_method == 3 && prec->table_bits < 2) { err = "Method 3 needs table_bits >= 2"; return MLMC_E_INVALID; }
    if (prec->packed) {
        if (estimator != MLMC_EST_APPROX) { err = "packed indices apply to APPROX only"; return MLMC_E_INVALID; }
        if (prec->arith != MLMC_ARITH_FP32 && prec->arith != MLMC_ARITH_FP16) { err = "packed indices need FP32 or FP16 arithmetic"; return MLMC_E_INVALID; }
        const int F = 32 / prec->table_bits;
        if (F != 4 && F != 5 && F != 8) { err = "packed indices need table_bits in {4, 6, 7, 8}"; return MLMC_E_INVALID; }
        if (prec->arith == MLMC_ARITH_FP16 && F != 4) { err = "packed FP16 indices need table_bits 7 or 8"; return MLMC_E_INVALID; }
    }
    if (prec->arith != MLMC_ARITH_FIXED) return MLMC_OK;
    const bool mil = p->scheme == MLMC_MILSTEIN;
    const int* w = prec->word_bits;
    const int* f = prec->frac_bits;
    for (int v = 0; v < MLMC_NVARS; ++v) {
        if (!fixed_vars_used(v, mil)) continue;
        const int wmax = v == MLMC_V_Z ? 31 : 32;
        if (w[v] < 2 || w[v] > wmax) { err = "word_bits out of range (2..32, Z 2..31) for variable " + std::to_string(v); return MLMC_E_INVALID; }
        if (f[v] < 0 || f[v] > 62) { err = "frac_bits out of range (0..62) for variable " + std::to_string(v); return MLMC_E_INVALID; }
    }
    // X_0 = 1 must be a value of X's format (the path starts there unsaturated)
    if (f[MLMC_V_X] > w[MLMC_V_X] - 2) { err = "X's format must hold 1: frac_bits[X] <= word_bits[X] - 2"; return MLMC_E_INVALID; }
    auto mul_ok = [&](int a, int b, int d) { return f[a] + f[b] - f[d] >= 0 && f[a] + f[b] - f[d] <= 62; };
    auto add_ok = [&](int a, int b, int d) {
        const int fm = std::max(f[a], f[b]);
        return std::abs(f[a] - f[b]) <= 30 && fm - f[d] >= 0 && fm - f[d] <= 62;
    };
    const int S = mil ? MLMC_V_SUM2 : MLMC_V_SUM1;
    bool ok = mul_ok(MLMC_V_X, S, MLMC_V_MUL2) && add_ok(MLMC_V_X, MLMC_V_MUL2, MLMC_V_X) &&
              mul_ok(MLMC_V_CON2, MLMC_V_Z, MLMC_V_MUL1) && add_ok(MLMC_V_CON1, MLMC_V_MUL1, MLMC_V_SUM1);
    if (mil) {
        ok = ok && mul_ok(MLMC_V_Z, MLMC_V_Z, MLMC_V_ZSQ) && f[MLMC_V_ZSQ] <= 30 &&
             add_ok(MLMC_V_ZSQ, MLMC_V_ZSQ, MLMC_V_ZM1) && mul_ok(MLMC_V_CON3, MLMC_V_ZM1, MLMC_V_MUL3) &&
             add_ok(MLMC_V_SUM1, MLMC_V_MUL3, MLMC_V_SUM2);
    }
    if (!ok) {
        err = "fixed-point formats: every product needs f_dst <= f_a + f_b, every sum f_dst <= max(f_a, f_b) "
              "and |f_a - f_b| <= 30 (zsq: f <= 30)";
        return MLMC_E_INVALID;
    }
    return MLMC_OK;
}

mlmc_status validate_all(const mlmc_problem* p, int32_t level, uint64_t n_paths, uint64_t path_offset,
                         const mlmc_precision* prec, int32_t estimator, std::string& err) {
    mlmc_status s = validate_problem(p, err);
    if (s != MLMC_OK) return s;
    if (level < 0 || level > 20) { err = "level must be 0..20"; return MLMC_E_INVALID; }
    if (estimator < MLMC_EST_PLAIN || estimator > MLMC_EST_CORR) { err = "estimator must be PLAIN, APPROX or CORR"; return MLMC_E_INVALID; }
    if (n_paths < 1) { err = "n_paths must be >= 1"; return MLMC_E_INVALID; }
    if (path_offset > (uint64_t(1) << 40) || n_paths > (uint64_t(1) << 40) - path_offset) { err = "path_offset + n_paths must be <= 2^40"; return MLMC_E_INVALID; }
    return validate_precision(prec, estimator, p, err);
}

// --------------------------------------------------------------- level prep
static FxOp mul_op(const int* f, const int* w, int a, int b, int d) {
    return fx_op_finish(FxOp{0, 0, f[a] + f[b] - f[d], w[d], 0, 0, 0, 0, 0});
}
static FxOp mul_op_fz(const int* f, const int* w, int fa, int fb, int d) {
    return fx_op_finish(FxOp{0, 0, fa + fb - f[d], w[d], 0, 0, 0, 0, 0});
}
static FxOp add_op(const int* f, const int* w, int fa, int fb, int d) {
    const int fm = std::max(fa, fb);
    return fx_op_finish(FxOp{fm - fa, fm - fb, fm - f[d], w[d], 0, 0, 0, 0, 0});
}

// Method 1's MSE E[(Z - T_q[k(Z)])^2] = 1 - 2^-q sum_k T_q[k]^2 (T_q[k] is the mean
// of Z on interval k, so the error is orthogonal to the table; Section 3.1).
double table_mse(int q) {
    const auto& T = method1_table(q);
    long double s = 0.0L;
    for (long double t : T) s += t * t;
    return static_cast<double>(1.0L - s / static_cast<long double>(uint64_t(1) << q));
}

// The largest |T_q[k]| (the end intervals' means).
double table_max_abs(int q) {
    const auto& T = method1_table(q);
    long double m = 0.0L;
    for (long double t : T) m = std::max(m, t < 0 ? -t : t);
    return static_cast<double>(m);
}

// The table values of (q, method) rounded once to FP32 (Method 1 from its exact
// interval means, Methods 2/3 from their FP64 values), kept for the process.
static const std::vector<float>& table_values_f32(int q, int method) {
    static std::map<std::pair<int, int>, std::vector<float>> cache;
    {
        std::lock_guard<std::mutex> lock(g_tables_mtx);
        auto it = cache.find({q, method});
        if (it != cache.end()) return it->second;
    }
    const uint32_t n = 1u << q;
    std::vector<float> v(n);
    if (method == 1) {
        const auto& T = method1_table(q);
        for (uint32_t k = 0; k < n; ++k) v[k] = static_cast<float>(T[k]);
    } else {
        const MethodTable& mt = method_table(q, method);
        for (uint32_t k = 0; k < n; ++k) v[k] = static_cast<float>(mt.z[k]);
    }
    std::lock_guard<std::mutex> lock(g_tables_mtx);
    return cache.emplace(std::make_pair(q, method), std::move(v)).first->second;
}

mlmc_status prepare_level(const mlmc_problem* p, int32_t level, const mlmc_precision* prec,
                          int32_t estimator, LevelPrep& out, std::string& err, bool with_table) {
    LevelDev& L = out.dev;
    std::memset(&L, 0, sizeof(L));
    const bool mil = p->scheme == MLMC_MILSTEIN;
    // constants in the order the method's reference computes them (FP64)
    const double h = p->T / static_cast<double>(uint64_t(1) << level);
    L.con1 = p->r * h;
    L.con1c = p->r * (2.0 * h);
    L.con2 = p->sigma * std::sqrt(h);
    L.con3 = ((0.5 * p->sigma) * p->sigma) * h;
    L.k = p->K / p->S0;
    L.b = p->barrier / p->S0;
    L.fcon1 = static_cast<float>(L.con1);
    L.fcon1c = static_cast<float>(L.con1c);
    L.fcon2 = static_cast<float>(L.con2);
    L.fcon3 = static_cast<float>(L.con3);
    L.f2con3 = static_cast<float>(2.0 * L.con3);
    L.fk = static_cast<float>(L.k);
    L.fb = static_cast<float>(L.b);
    if (prec->arith == MLMC_ARITH_FP16) {
        L.hcon1 = half_of(L.con1);
        L.hcon1c = half_of(L.con1c);
        L.hcon2 = half_of(L.con2);
        L.hcon3 = half_of(L.con3);
        L.hk = half_of(L.k);
        L.hb = half_of(L.b);
    }
    L.level = level;
    L.scheme = p->scheme;
    L.payoff_mask = p->payoff_mask;
    L.payoff_single = ctz32(p->payoff_mask);
    L.q = prec->table_bits;

    Variant& v = out.variant;
    v.est = estimator;
    v.arith = prec->arith;
    v.scheme = p->scheme;
    v.np = popcount32(p->payoff_mask) == 1 ? 1 : NPAY;
    v.track = ((p->payoff_mask >> MLMC_PAY_ASIAN) & 1u) || ((p->payoff_mask >> MLMC_PAY_BARRIER) & 1u);
    v.fields = (estimator == MLMC_EST_APPROX && prec->packed) ? 32 / prec->table_bits : 1;
    v.exact32 = estimator == MLMC_EST_CORR && prec->exact_side == 1;
    out.table.clear();
    if (estimator == MLMC_EST_PLAIN) return MLMC_OK;

    const int q = prec->table_bits;
    const uint32_t n = 1u << q;
    const int method = prec->rng_method > 1 ? prec->rng_method : 1;
    const MethodTable* mt = method == 1 ? nullptr : &method_table(q, method);
    // the values to tabulate, Method 1's exact interval means or Methods 2 / 3 in FP64
    // (the FP32 side takes them rounded once, from a per-(q, method) cache)
    std::vector<long double> Tm;
    const std::vector<long double>* Tp = nullptr;
    if (prec->arith != MLMC_ARITH_FP32 && with_table) {
        if (method == 1) {
            Tp = &method1_table(q);
        } else {
            Tm.resize(n);
            for (uint32_t k = 0; k < n; ++k) Tm[k] = mt->z[k];
            Tp = &Tm;
        }
    }
    const std::vector<long double>& T = Tp ? *Tp : Tm;
    L.table_entries = n;
    const bool needs_perm = mt && !mt->perm.empty() && estimator == MLMC_EST_CORR;
    if (!with_table && !needs_perm) {
        // the caller shares the bytes of an identical table (same arithmetic, q and
        // method); the constants are still this level's
        const size_t entry = prec->arith == MLMC_ARITH_FP16 ? 4 : 8;
        if (prec->arith == MLMC_ARITH_FIXED) {
            const int* f = prec->frac_bits;
            const int* w = prec->word_bits;
            L.fX = f[MLMC_V_X];
            L.wX = w[MLMC_V_X];
            L.icon1 = quantize_double(L.con1, f[MLMC_V_CON1], w[MLMC_V_CON1]);
            L.icon1c = quantize_double(L.con1c, f[MLMC_V_CON1], w[MLMC_V_CON1]);
            L.icon2 = quantize_double(L.con2, f[MLMC_V_CON2], w[MLMC_V_CON2]);
            L.icon3 = mil ? quantize_double(L.con3, f[MLMC_V_CON3], w[MLMC_V_CON3]) : 0;
            L.ik = quantize_double(L.k, f[MLMC_V_X], w[MLMC_V_X]);
            L.ib = quantize_double(L.b, f[MLMC_V_X], w[MLMC_V_X]);
            const int S = mil ? MLMC_V_SUM2 : MLMC_V_SUM1;
            L.op_mul2 = mul_op(f, w, MLMC_V_X, S, MLMC_V_MUL2);
            L.op_addX = add_op(f, w, f[MLMC_V_X], f[MLMC_V_MUL2], MLMC_V_X);
            L.op_mul1 = mul_op(f, w, MLMC_V_CON2, MLMC_V_Z, MLMC_V_MUL1);
            L.op_sum1 = add_op(f, w, f[MLMC_V_CON1], f[MLMC_V_MUL1], MLMC_V_SUM1);
            if (mil) {
                L.op_zsq = mul_op_fz(f, w, f[MLMC_V_Z], f[MLMC_V_Z], MLMC_V_ZSQ);
                L.op_zm1 = add_op(f, w, f[MLMC_V_ZSQ], f[MLMC_V_ZSQ], MLMC_V_ZM1);
                L.op_mul3 = mul_op(f, w, MLMC_V_CON3, MLMC_V_ZM1, MLMC_V_MUL3);
                L.op_sum2 = add_op(f, w, f[MLMC_V_SUM1], f[MLMC_V_MUL3], MLMC_V_SUM2);
                L.izm_c2 = int64_t(2) << f[MLMC_V_ZSQ];
            }
        }
        L.table_bytes = static_cast<uint32_t>((n * entry + 15) & ~size_t(15));
        return MLMC_OK;
    }
    if (prec->arith == MLMC_ARITH_FP32) {
        // (Z~_k, s_k): s_k is the fine step's multiplier of Z~_k, formed with the
        // same FP32 operations the kernels use on the coarse path
        const std::vector<float>& Z32 = table_values_f32(q, method);
        out.table.resize(static_cast<size_t>(n) * 8);
        for (uint32_t k = 0; k < n; ++k) {
            const float z = Z32[k];
            const float sf = mil ? multiplier32<true>(z, L.fcon1, L.fcon2, L.fcon3, 1.0f)
                                 : multiplier32<false>(z, L.fcon1, L.fcon2, L.fcon3, 1.0f);
            std::memcpy(&out.table[8 * k], &z, 4);
            std::memcpy(&out.table[8 * k + 4], &sf, 4);
        }
    } else if (prec->arith == MLMC_ARITH_FP16) {
        // (Z~_k, s_k) in binary16, s_k from the same FP16 operations as the kernels
        out.table.resize(static_cast<size_t>(n) * 4);
        for (uint32_t k = 0; k < n; ++k) {
            const _Float16 z = half_of(T[k]);
            const _Float16 one = 1;
            const _Float16 sh = mil ? multiplier_lp<true, _Float16>(z, L.hcon1, L.hcon2, L.hcon3, one)
                                    : multiplier_lp<false, _Float16>(z, L.hcon1, L.hcon2, L.hcon3, one);
            std::memcpy(&out.table[4 * k], &z, 2);
            std::memcpy(&out.table[4 * k + 2], &sh, 2);
        }
    } else {
        const int* f = prec->frac_bits;
        const int* w = prec->word_bits;
        L.fX = f[MLMC_V_X];
        L.wX = w[MLMC_V_X];
        L.icon1 = quantize_double(L.con1, f[MLMC_V_CON1], w[MLMC_V_CON1]);
        L.icon1c = quantize_double(L.con1c, f[MLMC_V_CON1], w[MLMC_V_CON1]);
        L.icon2 = quantize_double(L.con2, f[MLMC_V_CON2], w[MLMC_V_CON2]);
        L.icon3 = mil ? quantize_double(L.con3, f[MLMC_V_CON3], w[MLMC_V_CON3]) : 0;
        L.ik = quantize_double(L.k, f[MLMC_V_X], w[MLMC_V_X]);
        L.ib = quantize_double(L.b, f[MLMC_V_X], w[MLMC_V_X]);
        const int S = mil ? MLMC_V_SUM2 : MLMC_V_SUM1;
        L.op_mul2 = mul_op(f, w, MLMC_V_X, S, MLMC_V_MUL2);
        L.op_addX = add_op(f, w, f[MLMC_V_X], f[MLMC_V_MUL2], MLMC_V_X);
        L.op_mul1 = mul_op(f, w, MLMC_V_CON2, MLMC_V_Z, MLMC_V_MUL1);
        L.op_sum1 = add_op(f, w, f[MLMC_V_CON1], f[MLMC_V_MUL1], MLMC_V_SUM1);
        if (mil) {
            L.op_zsq = mul_op_fz(f, w, f[MLMC_V_Z], f[MLMC_V_Z], MLMC_V_ZSQ);
            L.op_zm1 = add_op(f, w, f[MLMC_V_ZSQ], f[MLMC_V_ZSQ], MLMC_V_ZM1);
            L.op_mul3 = mul_op(f, w, MLMC_V_CON3, MLMC_V_ZM1, MLMC_V_MUL3);
            L.op_sum2 = add_op(f, w, f[MLMC_V_SUM1], f[MLMC_V_MUL3], MLMC_V_SUM2);
            L.izm_c2 = int64_t(2) << f[MLMC_V_ZSQ];
        }
        out.table.resize(static_cast<size_t>(n) * 8);
        uint32_t nsat = 0;
        for (uint32_t k = 0; k < n; ++k) {
            int64_t z;
            if (!quantize_ld(T[k], f[MLMC_V_Z], w[MLMC_V_Z], z)) {
                err = "a table value does not fit Z's format";
                return MLMC_E_OVERFLOW;
            }
            // the fine step's multiplier, Algorithm 1's chain on Z~_k (with con1)
            const int64_t m1 = fx_mul(L.icon2, z, L.op_mul1, nsat);
            int64_t s = fx_add(L.icon1, m1, L.op_sum1, nsat);
            if (mil) {
                const int64_t zq = fx_mul(z, z, L.op_zsq, nsat);
                const int64_t zm = fx_add(zq, -(int64_t(1) << f[MLMC_V_ZSQ]), L.op_zm1, nsat);
                const int64_t m3 = fx_mul(L.icon3, zm, L.op_mul3, nsat);
                s = fx_add(s, m3, L.op_sum2, nsat);
            }
            const int32_t zi = static_cast<int32_t>(z), si = static_cast<int32_t>(s);
            std::memcpy(&out.table[8 * k], &zi, 4);
            std::memcpy(&out.table[8 * k + 4], &si, 4);
        }
        if (nsat) {
            err = "the fixed-point formats saturate in the table-driven part of the step (mul1/sum1/zsq/zm1/mul3/sum2 of some table value)";
            return MLMC_E_OVERFLOW;
        }
    }
    // Method 2's permutation for the exact side of the correction estimator
    if (needs_perm) {
        const size_t off = (out.table.size() + 15) & ~size_t(15);
        out.table.resize(off + 2 * static_cast<size_t>(n), 0);
        std::memcpy(&out.table[off], mt->perm.data(), 2 * static_cast<size_t>(n));
        L.perm_off = static_cast<uint32_t>(off);
    }
    L.table_bytes = static_cast<uint32_t>((out.table.size() + 15) & ~size_t(15));
    out.table.resize(L.table_bytes, 0);
    return MLMC_OK;
}

}  // namespace mlmc
