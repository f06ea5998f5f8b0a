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

// Inclusive prefix sum over the wave (every lane active) through DPP, with no LDS round trip: shifts
// by 1, 2, 4 and 8 lanes inside each row of 16 (a lane shifted in from outside the row adds 0), then
// rows 1 and 3 add the last lane of the row before them and rows 2 and 3 add lane 31.
__device__ __forceinline__ uint32_t plan_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t plan_sum_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)plan_incl_scan(v), 63);
}

__device__ __forceinline__ uint32_t plan_cls(const RepairSet* __restrict__ sets, uint32_t s, uint32_t which) {
    return repair_class(which ? (uint32_t)CT_HAMMING : sets[s].metric, sets[s].R);
}

// Parts per candidate of one set: gp of its class, at most one per min_sub boxes and eight per
// 64-box chunk (parts own box pb (mod 8) of chunk pc (mod parts / 8): more would idle), in whole
// eighths where there are 8 or more (part p of every candidate on XCD p mod 8), one for the
// enumerated classes.
__device__ __forceinline__ uint32_t plan_parts(const RepairSet& J, uint32_t cls, uint32_t gp, uint32_t min_sub) {
    const uint64_t pmax = min(J.n_sub / min_sub, ((J.n_sub + 63u) >> 6) * 8u);
    uint64_t p = gp > pmax ? pmax : gp;
    if (p >= 8) p &= ~7ull;
    if (p < 1 || cls / 4u == (uint32_t)CT_HAM1_RANDOM) p = 1;   // enumerated, not scanned
    return (uint32_t)p;
}

constexpr uint32_t kPlanCache = 4;   // sets per lane per slice of the plan

// One wave: per-set candidate counts -> parts and item offsets of one scan pass.  which = 0: main
// lists with each set's metric; which = 1: fallback lists, Hamming.  Each scan class is its own
// launch, so its candidates are split into parts to give that launch about target_items items,
// each part min_sub boxes or more.  The sets go in slices of 64 * per (per = min(kPlanCache,
// ceil(n_sets / 64))), lane l owning sets l * per .. l * per + per - 1 of a slice, whose class and
// list length stay in registers; every offset is a wave prefix (in set order) plus what earlier
// slices carried.  Only the classes in class_mask are visited, one at a time, class q's running
// figures held by lane q: a single wave issues this, so its instruction count is its duration.
__device__ inline void plan_wave(const RepairSet* __restrict__ sets, uint32_t n_sets, uint32_t which,
                                 const RepairPlan& plan, uint32_t class_mask, uint32_t target_items,
                                 uint32_t min_sub) {
    static_assert(kRepairClasses <= 64, "one lane per scan class");
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t per = min(kPlanCache, (n_sets + 63u) / 64u);
    const uint32_t slice_sets = 64u * per;
    const uint32_t slices = (n_sets + slice_sets - 1u) / slice_sets;
    uint32_t kc[kPlanCache], kn[kPlanCache];
    auto load = [&](uint32_t r) {
#pragma unroll
        for (uint32_t k = 0; k < kPlanCache; ++k) {
            const uint32_t s = r * slice_sets + lane * per + k;
            kc[k] = kRepairClasses;                    // no class: adds to nothing
            kn[k] = 0;
            if (k < per && s < n_sets) {
                kc[k] = plan_cls(sets, s, which);
                kn[k] = plan_count(sets, s, which);
            }
        }
    };
    // candidates per class (class q's total in lane q) -> parts per candidate of each class
    uint32_t tot = 0;
    for (uint32_t r = 0; r < slices; ++r) {
        load(r);
        for (uint32_t m = class_mask; m; m &= m - 1u) {
            const uint32_t q = (uint32_t)__builtin_ctz(m);
            uint32_t v = 0;
#pragma unroll
            for (uint32_t k = 0; k < kPlanCache; ++k) v += kc[k] == q ? kn[k] : 0u;
            const uint32_t t = plan_sum_u32(v);
            tot += lane == q ? t : 0u;
        }
    }
    const uint32_t gpc = tot ? max(target_items / tot, 1u) : 1u;
    uint32_t carry_c = 0;                              // candidates of earlier slices
    uint32_t carry = 0;                                // lane q: class q's items of earlier slices
    for (uint32_t r = 0; r < slices; ++r) {
        if (slices > 1) load(r);
        uint32_t kw[kPlanCache];
        uint32_t c_lane = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPlanCache; ++k) {
            const uint32_t s = r * slice_sets + lane * per + k;
            // parts per candidate of the set's class, from its lane (every lane takes part)
            const uint32_t gp = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(min(kc[k], 63u) * 4u), (int)gpc);
            kw[k] = 0;
            if (k < per && s < n_sets) {
                const uint32_t p = plan_parts(sets[s], kc[k], gp, min_sub);
                plan.parts[s] = p;
                kw[k] = kn[k] * p;
                c_lane += kn[k];
            }
        }
        const uint32_t ic = plan_incl_scan(c_lane);
        uint32_t oc = carry_c + ic - c_lane;
#pragma unroll
        for (uint32_t k = 0; k < kPlanCache; ++k) {
            const uint32_t s = r * slice_sets + lane * per + k;
            if (k < per && s < n_sets) {
                plan.cand_off[s] = oc;
                oc += kn[k];
            }
        }
        carry_c += (uint32_t)__builtin_amdgcn_readlane((int)ic, 63);
        for (uint32_t m = class_mask; m; m &= m - 1u) {
            const uint32_t q = (uint32_t)__builtin_ctz(m);
            uint32_t v = 0;
#pragma unroll
            for (uint32_t k = 0; k < kPlanCache; ++k) v += kc[k] == q ? kw[k] : 0u;
            const uint32_t iv = plan_incl_scan(v);
            uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)carry, (int)q) + iv - v;
#pragma unroll
            for (uint32_t k = 0; k < kPlanCache; ++k) {
                const uint32_t s = r * slice_sets + lane * per + k;
                if (k < per && s < n_sets) {
                    plan.item_off[q * (n_sets + 1) + s] = o;
                    o += kc[k] == q ? kw[k] : 0u;
                }
            }
            carry += lane == q ? (uint32_t)__builtin_amdgcn_readlane((int)iv, 63) : 0u;
        }
    }
    if (lane == 0) plan.cand_off[n_sets] = carry_c;
    if (lane < kRepairClasses && ((class_mask >> lane) & 1u)) plan.item_off[lane * (n_sets + 1) + n_sets] = carry;
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
