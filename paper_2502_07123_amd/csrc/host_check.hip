// The kernels' per-path code compiled for the host: a checker of the kernel
// arithmetic (records and sums) that runs without a GPU.  Groups are processed in
// order by one "thread", so per-path records equal the kernel's and sums differ
// from the kernel's only by FP64 summation order.
#include <cstring>
#include <string>

#include "device/paths.hpp"
#include "host/prepare.hpp"
#include "kernels.hpp"
#include "runtime.hpp"

namespace mlmc {
namespace {
struct HostGroups {
    const LevelDev* L;
    const WorkDev* W;
    const void* tab;
    bool buffered;                 // exact normals computed ahead (the runtime's default rule for a workspace of 192 MiB or more)
    SlotDev out{};
    template <class Tag>
    void operator()(Tag) {
        using B = PathBody<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track, Tag::fields, Tag::x32>;
        const uint64_t N = uint64_t(1) << L->level;
        const uint64_t S = group_span(L->level, B::WPB);
        const uint64_t G = S >> L->level;
        const uint64_t g0 = W->path_begin / G, g1 = (W->path_end - 1) / G + 1;
        Acc<Tag::np> acc;
        acc_zero(acc);
        if (B::HIST && L->level == 0) {
            std::vector<uint32_t> hist(L->table_entries, 0u);
            auto count = [&](uint32_t k) { hist[k] += 1u; };
            for (uint64_t g = g0; g < g1; ++g) B::hist_group(*L, *W, g, tab, count);
            for (uint32_t k = 0; k < L->table_entries; ++k)
                if (hist[k]) B::hist_accumulate(*L, tab, k, hist[k], acc);
        } else if (B::EX0 && L->level == 0 && !W->debug &&
                   uint32_t(Tag::np) * L->table_entries <= YTAB_MAX_ENTRIES) {
            // level 0 of the exact-normal estimators (no records), as the kernel runs it
            std::vector<double> yat(size_t(Tag::np) * L->table_entries, 0.0);
            if (B::HAS_TABLE)
                for (uint32_t k = 0; k < L->table_entries; ++k) B::ya_sample(*L, tab, k, yat.data());
            for (uint64_t g = g0; g < g1; ++g) B::exact0_group(*L, *W, g, tab, yat.data(), acc);
        } else if (B::HAS_EXACT && buffered) {
            // the buffered exact path: words and normals ahead, step-major, as k_normals
            using ZT = typename B::ExactT;
            const uint64_t P = W->path_end - W->path_begin, NN = uint64_t(1) << L->level;
            std::vector<uint32_t> Jb(P * NN);
            std::vector<ZT> Zb(P * NN);
            for (uint64_t b = (W->path_begin << L->level) / 4; b < (W->path_end << L->level) / 4; ++b) {
                const u32x4 r = philox4x32_10(u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32),
                                                    W->c2, W->c3}, W->k0, W->k1);
                const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
                for (int w = 0; w < 4; ++w) {
                    const uint64_t g = 4 * b + w;
                    const uint64_t idx = (g & (NN - 1)) * P + ((g >> L->level) - W->path_begin);
                    Jb[idx] = wd[w];
                    const uint32_t Je = B::coupled_word(*L, tab, wd[w]);
                    Zb[idx] = sizeof(ZT) == 4 ? static_cast<ZT>(norminv_f32(Je))
                                              : static_cast<ZT>(norminv_f64(Je));
                }
            }
            WorkDev W2 = *W;
            W2.jbuf = reinterpret_cast<uint64_t>(Jb.data());
            W2.zbuf = reinterpret_cast<uint64_t>(Zb.data());
            for (uint64_t i = W->path_begin; i < W->path_end; ++i) B::run_path_buffered(*L, W2, i, tab, acc);
        } else if ((B::FASTG || B::EXG) && L->level >= 1 && !W->debug) {
            for (uint64_t g = g0; g < g1; ++g) B::run_group_fast(*L, *W, g, tab, acc);
        } else {
            for (uint64_t g = g0; g < g1; ++g) B::run_group(*L, *W, g, tab, acc);
        }
        std::memset(&out, 0, sizeof(out));
        for (int p = 0; p < Tag::np; ++p) {
            out.s1[p] = acc.s1[p];
            out.s2[p] = acc.s2[p];
            out.e1[p] = acc.e1[p];
            out.e2[p] = acc.e2[p];
            out.i1[p] = acc.i1[p];
            out.i2lo[p] = acc.i2lo[p];
            out.i2hi[p] = acc.i2hi[p];
        }
        out.n = acc.n;
        out.sat = acc.sat;
        out.nonfinite = acc.nonfinite;
    }
};
}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" mlmc_status mlmc_check_paths_host(const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                                             uint64_t path_offset, const mlmc_precision* prec,
                                             int32_t estimator, uint64_t seed, uint32_t option_id,
                                             mlmc_sums* out, mlmc_path_record* records) {
    std::string err;
    mlmc_status s = validate_all(prob, level, n_paths, path_offset, prec, estimator, err);
    if (s != MLMC_OK) return s;
    if (!out || n_paths > 65536) return MLMC_E_INVALID;
    LevelPrep lp;
    s = prepare_level(prob, level, prec, estimator, lp, err);
    if (s != MLMC_OK) return s;
    WorkDev W;
    std::memset(&W, 0, sizeof(W));
    W.c2 = stream_c2(level, estimator);
    W.c3 = option_id;
    W.k0 = static_cast<uint32_t>(seed);
    W.k1 = static_cast<uint32_t>(seed >> 32);
    W.path_begin = path_offset;
    W.path_end = path_offset + n_paths;
    W.debug = reinterpret_cast<uint64_t>(records);
    const Tuning tune;
    const bool buffered = estimator != MLMC_EST_APPROX && level >= 2 && n_paths <= tune.zb_max_paths &&
                          (n_paths << level) <= tune.zb_max_positions;
    HostGroups h{&lp.dev, &W, lp.table.empty() ? nullptr : lp.table.data(), buffered};
    if (!dispatch_variant(lp.variant, h)) return MLMC_E_INVALID;
    const bool single = popcount32(prob->payoff_mask) == 1;
    int i = 0;
    for (int p = 0; p < MLMC_NPAYOFF; ++p)
        if ((prob->payoff_mask >> p) & 1u) slot_to_sums(h.out, single ? 0 : p, out[i++]);
    return MLMC_OK;
}
