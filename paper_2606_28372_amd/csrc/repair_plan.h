// Planning of one repair scan pass on the device: per-set candidate counts -> parts per
// candidate and item offsets per scan class.  Shared by the kernels that end in a plan (the
// proposal kernel, the repair preparation and the main pass's finish), whose last block to finish
// runs it, so that no launch of its own sits between them and the scans.
#pragma once

#include <hip/hip_runtime.h>

#include "ct_host.h"

// a set's list length, as the atomics that built it left it
__device__ __forceinline__ uint32_t plan_count(const RepairSet* __restrict__ sets, uint32_t s, uint32_t which) {
    return __hip_atomic_load(&sets[s].count[which], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t plan_excl_scan(uint32_t v, uint32_t lane) {
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x - v;
}

__device__ __forceinline__ uint32_t plan_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave: per-set candidate counts -> parts and item offsets of one scan pass.  Lane l owns
// a contiguous slice of the sets; offsets are the wave prefix of the lanes' totals plus the
// running sum inside the slice.  which = 0: main lists with each set's metric; which = 1:
// fallback lists, Hamming.  Each scan class is its own launch, so its candidates are split
// into parts to give that launch about target_items items, each part min_sub boxes or more, in a
// multiple of 8 parts where there are 8 or more (the scans place part p on XCD p mod 8).
__device__ inline void plan_wave(const RepairSet* __restrict__ sets, uint32_t n_sets, uint32_t which,
                                 const RepairPlan& plan, uint32_t class_mask, uint32_t target_items,
                                 uint32_t min_sub) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t chunk = (n_sets + 63u) / 64u;
    const uint32_t s0 = min(n_sets, lane * chunk), s1 = min(n_sets, s0 + chunk);
    uint32_t acc[kRepairClasses];
#pragma unroll
    for (uint32_t q = 0; q < kRepairClasses; ++q) acc[q] = 0;
    for (uint32_t s = s0; s < s1; ++s) {
        const uint32_t cls = repair_class(which ? (uint32_t)CT_HAMMING : sets[s].metric, sets[s].R);
        const uint32_t c = plan_count(sets, s, which);
#pragma unroll
        for (uint32_t q = 0; q < kRepairClasses; ++q) acc[q] += q == cls ? c : 0u;
    }
    uint32_t gpc[kRepairClasses];
#pragma unroll
    for (uint32_t q = 0; q < kRepairClasses; ++q) {
        gpc[q] = 1u;
        if (class_mask & (1u << q)) {
            const uint32_t total = plan_sum_u32(acc[q]);
            gpc[q] = total ? max(target_items / total, 1u) : 1u;
        }
    }
    uint32_t tc = 0;
#pragma unroll
    for (uint32_t q = 0; q < kRepairClasses; ++q) acc[q] = 0;
    for (uint32_t s = s0; s < s1; ++s) {
        // parts own box pb (mod 8) of chunk pc (mod parts / 8): more than 8 per chunk would idle
        const uint64_t pmax = min(sets[s].n_sub / min_sub, ((sets[s].n_sub + 63u) >> 6) * 8u);
        const uint32_t cls = repair_class(which ? (uint32_t)CT_HAMMING : sets[s].metric, sets[s].R);
        uint32_t gp = gpc[0];
#pragma unroll
        for (uint32_t q = 1; q < kRepairClasses; ++q) gp = q == cls ? gpc[q] : gp;
        uint64_t p = gp > pmax ? pmax : gp;
        if (p >= 8) p &= ~7ull;          // whole eighths: part p of every candidate on XCD p mod 8
        if (p < 1 || cls / 4u == (uint32_t)CT_HAM1_RANDOM) p = 1;   // enumerated, not scanned
        plan.parts[s] = (uint32_t)p;
        const uint32_t c = plan_count(sets, s, which);
        tc += c;
#pragma unroll
        for (uint32_t q = 0; q < kRepairClasses; ++q) acc[q] += q == cls ? c * (uint32_t)p : 0u;
    }
    uint32_t oc = plan_excl_scan(tc, lane);
#pragma unroll
    for (uint32_t q = 0; q < kRepairClasses; ++q)
        if (class_mask & (1u << q)) acc[q] = plan_excl_scan(acc[q], lane);
    for (uint32_t s = s0; s < s1; ++s) {
        const uint32_t p = plan.parts[s];
        const uint32_t c = plan_count(sets, s, which);
        const uint32_t cls = repair_class(which ? (uint32_t)CT_HAMMING : sets[s].metric, sets[s].R);
        plan.cand_off[s] = oc;
#pragma unroll
        for (uint32_t q = 0; q < kRepairClasses; ++q)
            if (class_mask & (1u << q)) plan.item_off[q * (n_sets + 1) + s] = acc[q];
        oc += c;
#pragma unroll
        for (uint32_t q = 0; q < kRepairClasses; ++q) acc[q] += q == cls ? c * p : 0u;
    }
    if (lane == 63) {
        plan.cand_off[n_sets] = oc;
#pragma unroll
        for (uint32_t q = 0; q < kRepairClasses; ++q)
            if (class_mask & (1u << q)) plan.item_off[q * (n_sets + 1) + n_sets] = acc[q];
    }
}


// What the last block of a kernel plans (enable = 0: nothing).
struct PlanArgs {
    RepairPlan plan;
    uint32_t class_mask, target_items, min_sub, which, enable;
};

// Called by every thread of every block at the end of a kernel whose results the plan reads (the
// sets' counters, only ever changed by atomics that return before the thread goes on): the last
// block to arrive runs the plan in its first wave and re-arms the counter.  No memory fence is
// needed (a device-scope fence writes back and invalidates the L2 of the block's XCD, which cost
// more than the launch it saves): the counters are read with device-scope atomic loads, which
// see every atomic already performed.  No thread may have left the kernel before this call.
__device__ inline void plan_if_last(const RepairSet* __restrict__ sets, uint32_t n_sets, const PlanArgs& pa) {
    if (!pa.enable) return;
    __shared__ uint32_t last;
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(pa.plan.done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!last) return;
    if (threadIdx.x < 64) plan_wave(sets, n_sets, pa.which, pa.plan, pa.class_mask, pa.target_items, pa.min_sub);
    if (threadIdx.x == 0) __hip_atomic_store(pa.plan.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
