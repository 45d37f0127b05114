// Device sweep engine kernels (engine.hpp): the driver's decisions per run, the
// device-side planning of a sweep's works and tiles, the fixed-order reduction of
// each work into its run's sums, and the upload of new runs and levels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device/advance.hpp"
#include "device/philox.hpp"
#include "device/reduce.hpp"
#include "engine.hpp"

namespace mlmc {

// One thread per slot: a run whose previous works have all been added gets its next
// works (or finishes).  Runs still holding works (not planned: a level not prepared
// yet, or no tile capacity) keep them.
__global__ void __launch_bounds__(64) k_eng_advance(EngPtrs p, uint32_t n_slots) {
    const uint32_t s = blockIdx.x * 64u + threadIdx.x;
    if (s >= n_slots) return;
    EngMeta& m = p.meta[s];
    if (!m.active || m.pending_valid) return;
    RunState& o = p.states[s];
    if (o.done) return;
    run_advance(o);
    m.pending_valid = o.n_pend > 0 ? 1u : 0u;
}

__device__ __forceinline__ WorkSplit eng_split(const EngHeader& H, const EngLevelInfo& in, int level,
                                               uint64_t begin, uint64_t n) {
    return split_groups(H.tile_steps, H.min_tiles, in.block, group_span(level, in.wpb), level, begin, n,
                        H.max_tiles_work);
}

constexpr uint32_t PLAN_THREADS = 1024;

// One block: the pending works of every run into per-class work lists.
//  1. per slot: are its works' levels prepared, its tiles in all; a prefix sum of
//     the tiles over the slots (in slot order) keeps the runs that fit the tile
//     slots (the rest wait for a later sweep);
//  2. per planned work: its place in its class's list and its first tile there, one
//     64-bit LDS atomic per work (place and tiles from one add, so the tile ranges
//     follow the places and the path kernels' tile search stays valid);
//  3. class offsets and counts (the path kernels read these);
//  4. per slot: work descriptors, tile descriptors and reduction entries, path
//     ranges continuing at the run's sample counts;
//  5. status words for the host.
// The order of works within a class may change from replay to replay; no result
// depends on it (a work's sums depend on its own tiles only, and a run adds at most
// one work per (level, estimator) per sweep).
__global__ void __launch_bounds__(PLAN_THREADS) k_eng_plan(EngPtrs p) {
    EngHeader& H = *p.hdr;
    const uint32_t C = H.n_slots, LV = H.n_levels, NC = H.n_classes;
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
    for (uint32_t base = 0; base < C; base += PLAN_THREADS) {
        const uint32_t s = base + tid;
        uint64_t total = 0;
        uint32_t planned = 0;
        if (s < C) {
            EngMeta& m = p.meta[s];
            uint32_t status = 0;
            if (m.active) {
                const RunState& o = p.states[s];
                if (o.done) status |= ENG_DONE;
                if (m.pending_valid) {
                    int need = -1;
                    for (int j = 0; j < o.n_pend; ++j)
                        if (o.pend[j].level >= static_cast<int>(m.levels_ready) && o.pend[j].level > need)
                            need = o.pend[j].level;
                    if (need >= 0) {
                        status |= ENG_WAIT_LEVEL | (static_cast<uint32_t>(need) << 8);
                    } else {
                        planned = 1;
                        for (int j = 0; j < o.n_pend; ++j) {
                            const int l = o.pend[j].level, e = o.pend[j].est;
                            const EngLevelInfo in = p.info[(s * LV + l) * 3u + e];
                            if (in.cls >= NC || in.block == 0 || in.wpb == 0) {   // never planned
                                H.error = 2u;
                                planned = 0;
                                break;
                            }
                            total += eng_split(H, in, l, o.sums[l][e].n, o.pend[j].n).nt;
                        }
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
        if (s < C) {
            p.scratch[s].planned = planned;
            p.scratch[s].total_tiles = total;
        }
        __syncthreads();
        if (tid == PLAN_THREADS - 1) carry += scan[tid];
        __syncthreads();
    }
    for (uint32_t s = tid; s < C; s += PLAN_THREADS) {
        EngPlanScratch& sc = p.scratch[s];
        if (!sc.planned) continue;
        const RunState& o = p.states[s];
        for (int j = 0; j < o.n_pend; ++j) {
            const int l = o.pend[j].level, e = o.pend[j].est;
            const EngLevelInfo in = p.info[(s * LV + l) * 3u + e];
            const uint64_t nt = eng_split(H, in, l, o.sums[l][e].n, o.pend[j].n).nt;
            const unsigned long long old = atomicAdd(&cls_acc[in.cls], (1ull << 32) | nt);
            sc.iw[j] = static_cast<uint32_t>(old >> 32);
            sc.t0[j] = static_cast<uint32_t>(old & 0xFFFFFFFFull);
        }
    }
    __syncthreads();
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
    for (uint32_t s = tid; s < C; s += PLAN_THREADS) {
        EngPlanScratch& sc = p.scratch[s];
        if (!sc.planned) continue;
        RunState& o = p.states[s];
        EngMeta& m = p.meta[s];
        for (int j = 0; j < o.n_pend; ++j) {
            const int l = o.pend[j].level, e = o.pend[j].est;
            const uint64_t n = o.pend[j].n;
            const EngLevelInfo in = p.info[(s * LV + l) * 3u + e];
            const uint32_t c = in.cls;
            const uint64_t begin = o.sums[l][e].n;
            const WorkSplit sp = eng_split(H, in, l, begin, n);
            const uint32_t gw = H.class_work_off[c] + sc.iw[j];
            const uint32_t t0 = sc.t0[j];
            WorkDev W;
            W.lvl = (s * LV + static_cast<uint32_t>(l)) * 3u + static_cast<uint32_t>(e);
            W.c2 = stream_c2(l, e);
            W.c3 = m.c3;
            W.k0 = m.k0;
            W.k1 = m.k1;
            W.pad0 = 0;
            W.path_begin = begin;
            W.path_end = begin + n;
            W.debug = 0;
            W.zbuf = 0;
            W.jbuf = 0;
            p.works[gw] = W;
            WorkTilesDev wt;
            wt.g0 = sp.g0;
            wt.g1 = sp.g1;
            wt.per = sp.per;
            wt.work = gw;
            wt.tile_end = t0 + static_cast<uint32_t>(sp.nt);
            wt.slot_begin = H.class_slot_off[c] + t0;
            wt.pad = 0;
            p.wtiles[gw] = wt;
            EngReduce rd;
            rd.slot_begin = wt.slot_begin;
            rd.slot_end = wt.slot_begin + static_cast<uint32_t>(sp.nt);
            rd.kind = in.kind;
            rd.run = s;
            rd.level = l;
            rd.est = e;
            rd.n = n;
            p.red[gw] = rd;
        }
        m.pending_valid = 0;
        o.sweeps += 1;
    }
    __syncthreads();
    for (uint32_t s = tid; s < C; s += PLAN_THREADS)
        p.status_out[s] = (p.meta[s].status & 0xFFFFu) | (p.meta[s].generation << 16);
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
        const SlotDev* sl = p.slots + rd.slot_begin;
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

// Uploads: block b copies segments b, b + grid, ... (system-scope loads: the staging
// buffer and the segment list are coherent pinned host memory).
__global__ void __launch_bounds__(256) k_eng_scatter(const uint8_t* __restrict__ staging,
                                                     const EngSeg* __restrict__ segs, uint32_t n) {
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint64_t* sp = reinterpret_cast<const uint64_t*>(segs + i);
        const uint64_t src = __hip_atomic_load(sp + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t dst = __hip_atomic_load(sp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t bytes = __hip_atomic_load(sp + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t* s = reinterpret_cast<const uint64_t*>(staging + src);
        uint64_t* d = reinterpret_cast<uint64_t*>(dst);
        for (uint64_t k = threadIdx.x; k < bytes / 8; k += 256)
            d[k] = __hip_atomic_load(s + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_eng_advance(const EngPtrs& p, uint32_t n_slots, hipStream_t st) {
    hipLaunchKernelGGL(k_eng_advance, dim3((n_slots + 63) / 64), dim3(64), 0, st, p, n_slots);
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
