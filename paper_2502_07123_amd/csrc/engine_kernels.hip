// Device sweep engine kernels (engine.hpp): the driver's decisions per run, the
// device-side planning of a sweep's works and tiles, the fixed-order reduction of
// each work into its run's sums, and the upload of new runs and levels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device/advance.hpp"
#include "device/philox.hpp"
#include "device/paths.hpp"
#include "device/reduce.hpp"
#include "engine.hpp"

namespace mlmc {

__device__ __forceinline__ WorkSplit eng_split(const EngHeader& H, const EngLevelInfo& in, int level,
                                               uint64_t begin, uint64_t n) {
    return split_groups(H.tile_steps, H.min_tiles, in.block, group_span(level, in.wpb), level, begin, n,
                        H.max_tiles_work);
}

// One block (one wave) per slot.  A run whose previous works have all been added
// gets its next works (or finishes); runs still holding works (not planned: a level
// not prepared yet, or no tile capacity) keep them.  The state is staged in LDS by
// the block (coalesced) and the decisions run on one lane against LDS.  Then, lane j
// per pending work j: its level's readiness, launch class and tile split into the
// slot's planning scratch, with the slot's totals.
constexpr uint32_t ADV_THREADS = 64;
static_assert(sizeof(RunState) % 8 == 0, "the state moves as 8-byte words");
static_assert(RUN_MAX_PEND <= ADV_THREADS, "one lane per pending work");

__global__ void __launch_bounds__(ADV_THREADS) k_eng_advance(EngPtrs p, uint32_t n_slots) {
    __shared__ RunState o;
    __shared__ uint32_t go, pend;
    __shared__ uint64_t nt_l[ADV_THREADS];
    __shared__ int32_t need_l[ADV_THREADS];
    __shared__ uint32_t bad_l[ADV_THREADS];
    const uint32_t s = blockIdx.x, tid = threadIdx.x;
    if (s >= n_slots) return;
    const EngHeader& H = *p.hdr;
    EngMeta& m = p.meta[s];
    if (tid == 0) {
        // 1: holds works, 2: may advance, 0: nothing to do (inactive or finished)
        go = !m.active ? 0u : (m.pending_valid ? 1u : (p.states[s].done ? 0u : 2u));
        pend = 0;
    }
    __syncthreads();
    if (!go) return;
    constexpr uint32_t NW = sizeof(RunState) / 8;
    const uint64_t* g = reinterpret_cast<const uint64_t*>(p.states + s);
    uint64_t* l = reinterpret_cast<uint64_t*>(&o);
    for (uint32_t k = tid; k < NW; k += ADV_THREADS) l[k] = g[k];
    __syncthreads();
    if (go == 2) {
        if (tid == 0) {
            run_advance(o);
            m.pending_valid = o.n_pend > 0 ? 1u : 0u;
            pend = o.n_pend > 0 ? 1u : 0u;
        }
        __syncthreads();
        uint64_t* gw = reinterpret_cast<uint64_t*>(p.states + s);
        for (uint32_t k = tid; k < NW; k += ADV_THREADS) gw[k] = l[k];
    } else if (tid == 0) {
        pend = 1;
    }
    __syncthreads();
    if (!pend) return;
    const uint32_t LV = H.n_levels, NC = H.n_classes;
    const int j = static_cast<int>(tid);
    uint64_t nt = 0;
    int32_t need = -1;
    uint32_t bad = 0;
    if (j < o.n_pend) {
        const int lv = o.pend[j].level, e = o.pend[j].est;
        if (lv >= static_cast<int>(m.levels_ready)) {
            need = lv;
        } else {
            const EngLevelInfo in = p.info[(s * LV + lv) * 3u + e];
            if (in.cls >= NC || in.block == 0 || in.wpb == 0) {
                bad = 1;
            } else {
                EngWorkPlan wp;
                wp.begin = o.sums[lv][e].n;
                wp.n = o.pend[j].n;
                wp.sp = eng_split(H, in, lv, wp.begin, wp.n);
                wp.level = lv;
                wp.est = e;
                wp.cls = in.cls;
                wp.kind = in.kind;
                wp.iw = wp.t0 = 0;
                p.scratch[s].w[j] = wp;
                nt = wp.sp.nt;
            }
        }
    }
    nt_l[tid] = nt;
    need_l[tid] = need;
    bad_l[tid] = bad;
    __syncthreads();
    if (tid == 0) {
        uint64_t t = 0;
        int32_t nd = -1;
        uint32_t bd = 0;
        for (uint32_t k = 0; k < ADV_THREADS; ++k) {
            t += nt_l[k];
            nd = need_l[k] > nd ? need_l[k] : nd;
            bd |= bad_l[k];
        }
        EngPlanScratch& sc = p.scratch[s];
        sc.total_tiles = t;
        sc.need = nd;
        sc.bad = bd;
        sc.n_works = static_cast<uint32_t>(o.n_pend);
    }
}

constexpr uint32_t PLAN_THREADS = 1024;

// One block: the pending works of every run into per-class work lists, from the
// planning scratch k_eng_advance wrote.  Phases over (slot, pending work) pairs run
// on all threads; phases over slots one thread per slot.
//  C. per slot: status; a prefix sum of the tiles over the slots (in slot order)
//     keeps the runs that fit the tile slots (the rest wait for a later sweep);
//  D. per planned work: its place in its class's list and its first tile there, one
//     64-bit LDS atomic per work (place and tiles from one add, so the tile ranges
//     follow the places and the path kernels' tile search stays valid);
//  E. class offsets and counts (the path kernels read these);
//  F. per planned work: work descriptor, tile descriptor and reduction entry;
//  G. per slot: the works handed over; status words for the host.
// The order of works within a class may change from replay to replay; no result
// depends on it (a work's sums depend on its own tiles only, and a run adds at most
// one work per (level, estimator) per sweep).
__global__ void __launch_bounds__(PLAN_THREADS) k_eng_plan(EngPtrs p) {
    EngHeader& H = *p.hdr;
    const uint32_t C = H.n_slots, LV = H.n_levels, NC = H.n_classes;
    const uint32_t NI = C * static_cast<uint32_t>(RUN_MAX_PEND);
    const uint32_t tid = threadIdx.x;
    __shared__ unsigned long long cls_acc[ENG_MAX_CLASSES];   // works << 32 | tiles
    __shared__ uint64_t scan[PLAN_THREADS];
    __shared__ uint64_t carry;
    __shared__ uint32_t n_planned, n_deferred;
    if (tid < ENG_MAX_CLASSES) cls_acc[tid] = 0ull;
    if (tid == 0) {
        carry = 0;
        n_planned = n_deferred = 0;
    }
    __syncthreads();
    // C
    for (uint32_t base = 0; base < C; base += PLAN_THREADS) {
        const uint32_t s = base + tid;
        uint64_t total = 0;
        uint32_t planned = 0;
        if (s < C) {
            EngMeta& m = p.meta[s];
            const EngPlanScratch& sc = p.scratch[s];
            uint32_t status = 0;
            if (m.active) {
                if (p.states[s].done) status |= ENG_DONE;
                if (m.pending_valid) {
                    if (sc.need >= 0) {
                        status |= ENG_WAIT_LEVEL | (static_cast<uint32_t>(sc.need) << 8);
                    } else if (sc.bad) {
                        H.error = 2u;                                      // never planned
                    } else {
                        planned = 1;
                        total = sc.total_tiles;
                    }
                }
            }
            m.status = status;
        }
        scan[tid] = planned ? total : 0;
        __syncthreads();
        for (uint32_t off = 1; off < PLAN_THREADS; off <<= 1) {
            const uint64_t v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        if (planned && carry + scan[tid] > H.slot_cap) {
            if (total > H.slot_cap) H.error = 1u;
            planned = 0;
            atomicAdd(&n_deferred, 1u);
        }
        if (planned) atomicAdd(&n_planned, 1u);
        if (s < C) p.scratch[s].planned = planned;
        __syncthreads();
        if (tid == PLAN_THREADS - 1) carry += scan[tid];
        __syncthreads();
    }
    // D
    for (uint32_t idx = tid; idx < NI; idx += PLAN_THREADS) {
        const uint32_t s = idx / static_cast<uint32_t>(RUN_MAX_PEND);
        const uint32_t j = idx % static_cast<uint32_t>(RUN_MAX_PEND);
        EngPlanScratch& sc = p.scratch[s];
        if (!sc.planned || j >= sc.n_works) continue;
        EngWorkPlan& w = sc.w[j];
        const unsigned long long old = atomicAdd(&cls_acc[w.cls], (1ull << 32) | w.sp.nt);
        w.iw = static_cast<uint32_t>(old >> 32);
        w.t0 = static_cast<uint32_t>(old & 0xFFFFFFFFull);
    }
    __syncthreads();
    // E
    if (tid == 0) {
        uint32_t ow = 0, ot = 0;
        for (uint32_t c = 0; c < NC; ++c) {
            const uint32_t w = static_cast<uint32_t>(cls_acc[c] >> 32);
            const uint32_t t = static_cast<uint32_t>(cls_acc[c] & 0xFFFFFFFFull);
            H.class_work_off[c] = ow;
            H.class_slot_off[c] = ot;
            H.counts[c][0] = w;
            H.counts[c][1] = t;
            H.counts[c][2] = ow;
            H.counts[c][3] = 0;
            ow += w;
            ot += t;
        }
        H.n_works = ow;
        H.planned = n_planned;
        H.deferred = n_deferred;
    }
    __syncthreads();
    // F
    for (uint32_t idx = tid; idx < NI; idx += PLAN_THREADS) {
        const uint32_t s = idx / static_cast<uint32_t>(RUN_MAX_PEND);
        const uint32_t j = idx % static_cast<uint32_t>(RUN_MAX_PEND);
        const EngPlanScratch& sc = p.scratch[s];
        if (!sc.planned || j >= sc.n_works) continue;
        const EngWorkPlan w = sc.w[j];
        const EngMeta& m = p.meta[s];
        const uint32_t c = w.cls;
        const uint32_t gw = H.class_work_off[c] + w.iw;
        WorkDev W;
        W.lvl = (s * LV + static_cast<uint32_t>(w.level)) * 3u + static_cast<uint32_t>(w.est);
        W.c2 = stream_c2(w.level, w.est);
        W.c3 = m.c3;
        W.k0 = m.k0;
        W.k1 = m.k1;
        W.pad0 = 0;
        W.path_begin = w.begin;
        W.path_end = w.begin + w.n;
        W.debug = 0;
        W.zbuf = 0;
        W.jbuf = 0;
        p.works[gw] = W;
        WorkTilesDev wt;
        wt.g0 = w.sp.g0;
        wt.g1 = w.sp.g1;
        wt.per = w.sp.per;
        wt.work = gw;
        wt.tile_end = w.t0 + static_cast<uint32_t>(w.sp.nt);
        wt.slot_begin = H.class_slot_off[c] + w.t0;
        wt.pad = 0;
        p.wtiles[gw] = wt;
        EngReduce rd;
        rd.slot_begin = wt.slot_begin;
        rd.slot_end = wt.slot_begin + static_cast<uint32_t>(w.sp.nt);
        rd.kind = w.kind;
        rd.run = s;
        rd.level = w.level;
        rd.est = w.est;
        rd.n = w.n;
        p.red[gw] = rd;
    }
    __syncthreads();
    // G
    for (uint32_t s = tid; s < C; s += PLAN_THREADS) {
        if (p.scratch[s].planned) {
            p.meta[s].pending_valid = 0;
            p.states[s].sweeps += 1;
        }
        p.status_out[s] = (p.meta[s].status & 0xFFFFu) | (p.meta[s].generation << 16);
    }
    if (tid == 0) p.status_out[C] = H.error;
}

// Each work's tile slots in the fixed order (reduce_work, as the launch sequences'
// k_reduce), then added into its run's sums; the run's sample count advances with
// the sums (the next path index of the stream).
__global__ void __launch_bounds__(REDUCE_THREADS) k_eng_reduce(EngPtrs p) {
    __shared__ RedLds red;
    __shared__ SlotDev res;
    const uint32_t nw = p.hdr->n_works;
    for (uint32_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const EngReduce rd = p.red[w];
        const TileSlot* sl = p.slots + rd.slot_begin;
        const uint32_t ns = rd.slot_end - rd.slot_begin;
        switch (rd.kind & 3u) {
            case 1: reduce_work<1, true, false>(sl, ns, &res, red); break;
            case 2: reduce_work<1, false, true>(sl, ns, &res, red); break;
            default: reduce_work<1, false, false>(sl, ns, &res, red); break;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            EstSums b;
            b.n = res.n;
            b.s1 = res.s1[0];
            b.s2 = res.s2[0];
            b.e1 = res.e1[0];
            b.e2 = res.e2[0];
            b.i1 = res.i1[0];
            b.i2lo = res.i2lo[0];
            b.i2hi = res.i2hi[0];
            b.sat = res.sat;
            b.nonfinite = res.nonfinite;
            RunState& o = p.states[rd.run];
            est_accumulate(o.sums[rd.level][rd.est], b);
            atomicAdd(reinterpret_cast<unsigned long long*>(&o.path_steps),
                      static_cast<unsigned long long>(rd.n << rd.level));
        }
        __syncthreads();
    }
}

// Uploads: block b copies segments b, b + grid, ... from the device staging area
// (filled by a DMA copy from pinned host memory) or writes zeros.
__global__ void __launch_bounds__(256) k_eng_scatter(const uint8_t* __restrict__ staging,
                                                     const EngSeg* __restrict__ segs, uint32_t n) {
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const EngSeg g = segs[i];
        uint64_t* d = reinterpret_cast<uint64_t*>(g.dst);
        const uint64_t nw = g.bytes / 8;
        if (g.src == ENG_SEG_ZERO) {
            for (uint64_t k = threadIdx.x; k < nw; k += 256) d[k] = 0;
        } else {
            const uint64_t* s = reinterpret_cast<const uint64_t*>(staging + g.src);
            for (uint64_t k = threadIdx.x; k < nw; k += 256) d[k] = s[k];
        }
    }
}

// One block per job; entries k = tid, tid + 256, ... of the level's 2^q.
__global__ void __launch_bounds__(256) k_eng_tables(const EngTableJob* __restrict__ jobs, const LevelDev* levels,
                                                    const uint8_t* __restrict__ base, uint8_t* tables) {
    const EngTableJob j = jobs[blockIdx.x];
    const LevelDev& L = levels[j.lvl];
    const uint32_t n = L.table_entries;
    if (j.arith == MLMC_ARITH_FP32) {
        const float* z = reinterpret_cast<const float*>(base + j.base_off);
        float* t = reinterpret_cast<float*>(tables + j.table_off);
        for (uint32_t k = threadIdx.x; k < n; k += 256) {
            const float zk = z[k];
            t[2 * k] = zk;
            t[2 * k + 1] = j.mil ? multiplier32<true>(zk, L.fcon1, L.fcon2, L.fcon3, 1.0f)
                                 : multiplier32<false>(zk, L.fcon1, L.fcon2, L.fcon3, 1.0f);
        }
    } else {
        const _Float16* z = reinterpret_cast<const _Float16*>(base + j.base_off);
        _Float16* t = reinterpret_cast<_Float16*>(tables + j.table_off);
        const _Float16 one = 1;
        for (uint32_t k = threadIdx.x; k < n; k += 256) {
            const _Float16 zk = z[k];
            t[2 * k] = zk;
            t[2 * k + 1] = j.mil ? multiplier_lp<true, _Float16>(zk, L.hcon1, L.hcon2, L.hcon3, one)
                                 : multiplier_lp<false, _Float16>(zk, L.hcon1, L.hcon2, L.hcon3, one);
        }
    }
}

hipError_t launch_eng_tables(const EngTableJob* jobs, uint32_t n, const LevelDev* levels, const uint8_t* base,
                             uint8_t* tables, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eng_tables, dim3(n), dim3(256), 0, st, jobs, levels, base, tables);
    return hipGetLastError();
}

hipError_t launch_eng_advance(const EngPtrs& p, uint32_t n_slots, hipStream_t st) {
    hipLaunchKernelGGL(k_eng_advance, dim3(n_slots), dim3(ADV_THREADS), 0, st, p, n_slots);
    return hipGetLastError();
}

hipError_t launch_eng_plan(const EngPtrs& p, hipStream_t st) {
    hipLaunchKernelGGL(k_eng_plan, dim3(1), dim3(PLAN_THREADS), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_eng_reduce(const EngPtrs& p, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_eng_reduce, dim3(grid), dim3(REDUCE_THREADS), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_eng_scatter(const uint8_t* staging, const EngSeg* segs, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eng_scatter, dim3(n < 1024 ? n : 1024), dim3(256), 0, st, staging, segs, n);
    return hipGetLastError();
}

}  // namespace mlmc
