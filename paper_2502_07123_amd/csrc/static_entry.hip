// mlmc_level_sums_static: the level sums of one (level, estimator) path range with
// no allocation of any kind on the device side, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The plan (level constants, the work, its tile descriptor and reduction entry,
// the step table) and the per-tile partial sums live in `scratch`, a file-scope
// device array of SCRATCH_BYTES per GPU.  Its device address is looked up once
// per device with hipGetSymbolAddress (the array's name in host code is only a
// host-side stand-in) and that address is what the kernels receive.  The plan
// travels as kernel arguments (k_put, in chunks), so no staging memory is needed
// either; the path kernel and the fixed-order reduction are the library's own,
// with the same tile split as mlmc_level_sums, so the sums are the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "device/philox.hpp"
#include "runtime.hpp"

namespace mlmc {

// 4 MiB per GPU: the plan (under 48 KiB with the largest table) and up to
// STATIC_MAX_TILES tile partials of 384 bytes (3 MiB).
constexpr size_t SCRATCH_BYTES = size_t(4) << 20;
constexpr uint64_t STATIC_MAX_TILES = 8192;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

// One chunk of the plan carried by value as kernel arguments (a ~2 KiB kernarg
// segment) and stored at byte offset off of the scratch array.
constexpr uint32_t PUT_WORDS = 248;
struct PutChunk {
    uint32_t off;       // byte offset (multiple of 8)
    uint32_t n;         // 8-byte words in w
    uint64_t w[PUT_WORDS];
};

__global__ void __launch_bounds__(256) k_put(uint8_t* __restrict__ base, PutChunk c) {
    uint64_t* dst = reinterpret_cast<uint64_t*>(base + c.off);
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

// The work's sums in the ABI's layout: out[j] for the j-th payoff bit of mask
// (slot 0 for a one-payoff kernel, slot p otherwise).
__global__ void k_sums_out(const SlotDev* __restrict__ res, uint32_t mask, mlmc_sums* __restrict__ out) {
    if (threadIdx.x != 0) return;
    const SlotDev& s = *res;
    const bool single = (mask & (mask - 1u)) == 0u;
    int j = 0;
    for (int p = 0; p < NPAY; ++p) {
        if (!((mask >> p) & 1u)) continue;
        const int i = single ? 0 : p;
        mlmc_sums o;
        o.n = s.n;
        o.sum1 = s.s1[i];
        o.sum2 = s.s2[i];
        o.isum1 = s.i1[i];
        o.isum2_lo = s.i2lo[i];
        o.isum2_hi = s.i2hi[i];
        o.esum1 = s.e1[i];
        o.esum2 = s.e2[i];
        o.saturations = s.sat;
        o.nonfinite = s.nonfinite;
        out[j++] = o;
    }
}

namespace {

constexpr int MAX_DEVICES = 64;

// Per device: the scratch array's device address and the CU count, set once with
// that device current.
struct StaticDevice {
    std::once_flag once;
    hipError_t err = hipSuccess;
    uint8_t* ptr = nullptr;
    int cus = 0;
};
StaticDevice g_static[MAX_DEVICES];

thread_local std::string t_static_err;

mlmc_status static_fail(mlmc_status s, const std::string& msg) {
    t_static_err = msg;
    return s;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

hipError_t put_bytes(uint8_t* base, size_t off, const void* src, size_t bytes, hipStream_t st) {
    const uint8_t* p = static_cast<const uint8_t*>(src);
    PutChunk c;
    for (size_t done = 0; done < bytes;) {
        const size_t take = std::min(bytes - done, sizeof(c.w));
        std::memset(c.w, 0, sizeof(c.w));
        std::memcpy(c.w, p + done, take);
        c.off = static_cast<uint32_t>(off + done);
        c.n = static_cast<uint32_t>((take + 7) / 8);
        hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, base, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done += take;
    }
    return hipSuccess;
}

}  // namespace

const char* static_last_error() { return t_static_err.c_str(); }

}  // namespace mlmc

using namespace mlmc;

extern "C" mlmc_status mlmc_level_sums_static(const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                                              uint64_t path_offset, const mlmc_precision* prec,
                                              int32_t estimator, uint64_t seed, uint32_t option_id,
                                              void* stream, mlmc_sums* out_dev) {
    std::string err;
    mlmc_status s = validate_all(prob, level, n_paths, path_offset, prec, estimator, err);
    if (s != MLMC_OK) return static_fail(s, err);
    if (!out_dev) return static_fail(MLMC_E_INVALID, "out_dev is NULL");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return static_fail(MLMC_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return static_fail(MLMC_E_INVALID, "device index out of range");
    StaticDevice& sd = g_static[dev];
    std::call_once(sd.once, [&sd, dev]() {
        void* p = nullptr;
        sd.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (sd.err == hipSuccess) sd.ptr = static_cast<uint8_t*>(p);
        if (sd.err == hipSuccess) sd.err = hipDeviceGetAttribute(&sd.cus, hipDeviceAttributeMultiprocessorCount, dev);
    });
    if (sd.err != hipSuccess || !sd.ptr)
        return static_fail(MLMC_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(sd.err));

    // the level (constants, step table, kernel variant) and the launch geometry
    LevelPrep lp;
    s = prepare_level(prob, level, prec, estimator, lp, err);
    if (s != MLMC_OK) return static_fail(s, err);
    const VariantInfo vi = variant_info(lp.variant);
    if (!vi.fn) return static_fail(MLMC_E_INVALID, "no compiled kernel for this estimator/arithmetic/packing");
    const Tuning tune;                                     // the library's default geometry
    const uint32_t block = block_for(tune, lp.variant, vi);
    const uint64_t S = group_span(level, static_cast<uint32_t>(vi.wpb));
    const WorkSplit sp = split_work(tune, block, S, level, path_offset, n_paths, STATIC_MAX_TILES);
    const uint32_t lds = lds_bytes_for(lp.variant, lp.dev);

    // layout: [result | level | work | work tiles | reduction | counts | table | tile slots]
    const size_t o_res = 0;
    const size_t o_lvl = align256(o_res + sizeof(SlotDev));
    const size_t o_work = align256(o_lvl + sizeof(LevelDev));
    const size_t o_tile = align256(o_work + sizeof(WorkDev));
    const size_t o_red = align256(o_tile + sizeof(WorkTilesDev));
    const size_t o_cnt = align256(o_red + sizeof(ReduceDev));
    const size_t o_tab = align256(o_cnt + 4 * sizeof(uint32_t));
    const size_t o_slot = align256(o_tab + lp.table.size());
    const size_t need = o_slot + sp.nt * sizeof(TileSlot);
    if (sp.nt > STATIC_MAX_TILES || need > SCRATCH_BYTES)
        return static_fail(MLMC_E_NOMEM, "mlmc_level_sums_static: needs " + std::to_string(need) +
                                             " bytes of its " + std::to_string(SCRATCH_BYTES) + "-byte scratch");

    LevelDev L = lp.dev;
    L.table_off = 0;                                      // tables pointer = the table itself
    WorkDev W;
    std::memset(&W, 0, sizeof(W));
    W.lvl = 0;
    W.c2 = stream_c2(level, estimator);
    W.c3 = option_id;
    W.k0 = static_cast<uint32_t>(seed);
    W.k1 = static_cast<uint32_t>(seed >> 32);
    W.path_begin = path_offset;
    W.path_end = path_offset + n_paths;
    WorkTilesDev wt;
    std::memset(&wt, 0, sizeof(wt));
    wt.g0 = sp.g0;
    wt.g1 = sp.g1;
    wt.per = sp.per;
    wt.work = 0;
    wt.tile_end = static_cast<uint32_t>(sp.nt);
    wt.slot_begin = 0;
    ReduceDev rd;
    rd.slot_begin = 0;
    rd.slot_end = static_cast<uint32_t>(sp.nt);
    rd.kind = (estimator == MLMC_EST_CORR ? 1u : 0u) |
              (estimator == MLMC_EST_APPROX && prec->arith == MLMC_ARITH_FIXED ? 2u : 0u) |
              (lp.variant.np == NPAY ? 4u : 0u);
    rd.work = 0;

    // one host buffer [level .. table] on the stack, sent as kernel arguments
    uint8_t plan[align256(sizeof(LevelDev)) + align256(sizeof(WorkDev)) + align256(sizeof(WorkTilesDev)) +
                 align256(sizeof(ReduceDev)) + 256];
    if (o_tab - o_lvl > sizeof(plan)) return static_fail(MLMC_E_INVALID, "plan header layout");
    std::memset(plan, 0, sizeof(plan));
    std::memcpy(plan + (o_lvl - o_lvl), &L, sizeof(L));
    std::memcpy(plan + (o_work - o_lvl), &W, sizeof(W));
    std::memcpy(plan + (o_tile - o_lvl), &wt, sizeof(wt));
    std::memcpy(plan + (o_red - o_lvl), &rd, sizeof(rd));
    const uint32_t counts[4] = {1u, static_cast<uint32_t>(sp.nt), 0u, 0u};  // work descriptors, tiles
    std::memcpy(plan + (o_cnt - o_lvl), counts, sizeof(counts));

    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* d = sd.ptr;
    e = put_bytes(d, o_lvl, plan, o_tab - o_lvl, st);
    if (e == hipSuccess && !lp.table.empty()) e = put_bytes(d, o_tab, lp.table.data(), lp.table.size(), st);
    if (e != hipSuccess) return static_fail(MLMC_E_DEVICE, std::string("plan: ") + hipGetErrorString(e));
    const uint32_t grid = static_cast<uint32_t>(
        std::min<uint64_t>(sp.nt, uint64_t(std::max(1, sd.cus)) * tune.blocks_per_cu));
    e = launch_paths(vi, grid, block, lds, st, reinterpret_cast<const WorkTilesDev*>(d + o_tile),
                     reinterpret_cast<const uint32_t*>(d + o_cnt), reinterpret_cast<const WorkDev*>(d + o_work),
                     reinterpret_cast<const LevelDev*>(d + o_lvl), d + o_tab,
                     reinterpret_cast<TileSlot*>(d + o_slot));
    if (e == hipSuccess)
        e = launch_reduce(1, st, reinterpret_cast<const TileSlot*>(d + o_slot),
                          reinterpret_cast<const ReduceDev*>(d + o_red), reinterpret_cast<SlotDev*>(d + o_res));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sums_out, dim3(1), dim3(64), 0, st, reinterpret_cast<const SlotDev*>(d + o_res),
                           prob->payoff_mask, out_dev);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return static_fail(MLMC_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return MLMC_OK;
}
