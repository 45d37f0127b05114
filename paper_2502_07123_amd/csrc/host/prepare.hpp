// Host-side preparation of launches (internal): validation, per-level constants,
// Method-1 tables and step tables, kernel variant choice.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../common.hpp"
#include "../kernels.hpp"

namespace mlmc {

// Method-1 table T_q in long double (cached per q).
const std::vector<long double>& method1_table(int q);

// Table values of Methods 2 (n = 2) and 3 of Section 3 in FP64, and Method 2's
// permutation pi (empty for Method 3); cached per (q, method).
struct MethodTable {
    std::vector<double> z;
    std::vector<uint16_t> perm;
    int iterations = 0;
};
const MethodTable& method_table(int q, int method);

// Round T_q into the storage format of mlmc_build_table.
mlmc_status build_table_bytes(int q, int arith, int frac_bits, void* out, std::string& err);

// Validation shared by every entry point; err receives the reason.
mlmc_status validate_problem(const mlmc_problem* p, std::string& err);
mlmc_status validate_precision(const mlmc_precision* prec, int estimator, const mlmc_problem* p,
                               std::string& err);
mlmc_status validate_all(const mlmc_problem* p, int32_t level, uint64_t n_paths,
                         uint64_t path_offset, const mlmc_precision* prec, int32_t estimator,
                         std::string& err);

// Everything a launch needs for one (problem, level, precision, estimator).
struct LevelPrep {
    LevelDev dev;                  // table_off filled in by the planner
    std::vector<uint8_t> table;    // step table bytes (empty: none)
    Variant variant;
};

// Builds constants, the step table and the variant.  MLMC_E_OVERFLOW when a
// fixed-point table entry saturates (the table-driven part must be exact).
// with_table false: no table bytes (table_bytes still set) unless the estimator's
// table differs from the approximate estimator's of the same precision (Method 2's
// correction table carries the permutation) -- for callers that share that table.
mlmc_status prepare_level(const mlmc_problem* p, int32_t level, const mlmc_precision* prec,
                          int32_t estimator, LevelPrep& out, std::string& err, bool with_table = true);

int popcount32(uint32_t v);

// Method 1 table statistics (Section 3.1): its MSE and its largest |value|.
double table_mse(int q);
double table_max_abs(int q);

}  // namespace mlmc
