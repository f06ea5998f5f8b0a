// ct_repair_noalloc: the repair of ct_repair (same kernels, same results) for callers that
// cannot allocate device memory -- code under stream capture, tight serving loops, harnesses
// that forbid the allocator.  Its scratch (candidate lists, per-part winners, the candidate set
// descriptor and the scan plan) lives in one file-scope device array instead of a per-call
// allocation.  Each GPU holds its own copy of the array until the process ends; host code never
// uses the array's name as an address (on the host it is only a stand-in symbol): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ct_host.h"
#include "repair_plan.h"

namespace {

// Layout of the scratch array for at most CT_NOALLOC_MAX_ROWS candidates, fixed offsets.
constexpr uint64_t kRows = CT_NOALLOC_MAX_ROWS;
constexpr uint64_t kSlots = kRows > kRepairTargetWaves ? kRows : kRepairTargetWaves;
constexpr uint64_t kPlanWords = 2ull * (1 + kRepairClasses) + 1 + 1;   // one set: cand_off, item_off, parts, done
constexpr uint64_t align8(uint64_t x) { return (x + 7) & ~7ull; }
constexpr uint64_t kOffList = 0;
constexpr uint64_t kOffListIns = kOffList + align8(kRows * 4);
constexpr uint64_t kOffFbList = kOffListIns + kRows * 8;
constexpr uint64_t kOffFbIns = kOffFbList + align8(kRows * 4);
constexpr uint64_t kOffPartKey = kOffFbIns + kRows * 8;
constexpr uint64_t kOffPartPos = kOffPartKey + kSlots * 8;
constexpr uint64_t kOffCount = kOffPartPos + align8(kSlots * 4);
constexpr uint64_t kOffPrep = kOffCount + 8;
constexpr uint64_t kOffPlan = kOffPrep + 8;
constexpr uint64_t kOffSet = (kOffPlan + kPlanWords * 4 + 255) & ~255ull;
constexpr uint64_t kScratchBytes = kOffSet + ((sizeof(RepairSet) + 255) & ~255ull);
static_assert(kScratchBytes <= CT_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds the documented size");

}  // namespace

static __device__ __align__(256) uint8_t scratch[CT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (null: not looked up)

// The array's address on the current device, looked up on the first call there.
int scratch_on_current_device(int dev, uint8_t** out) {
    if (dev < 0 || dev >= kMaxDevices) return ct_fail(CT_EINVAL, "ct_repair_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return ct_fail(CT_EDEVICE, std::string("ct_repair_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch[dev];
    return CT_OK;
}

// Writes the candidate set descriptor into the scratch and clears what must start at zero (the
// list counters and the plan's block counter), so nothing here is a memset or a host copy.
__global__ void k_noalloc_setup(RepairSet h, RepairSet* __restrict__ d_set, uint32_t* __restrict__ prep_off,
                                uint32_t* __restrict__ plan_done) {
    if (threadIdx.x == 0) {
        *d_set = h;
        h.count[0] = 0;
        h.count[1] = 0;
        prep_off[0] = 0;
        prep_off[1] = h.n;
        *plan_done = 0;
    }
}

}  // namespace

extern "C" int ct_repair_noalloc(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric, uint64_t seed,
                                 uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16,
                                 uint8_t* d_out_rows, uint32_t* d_out_pos, void* stream) {
    if (!s || (n && (!d_rows || !d_out_rows || !d_out_pos)))
        return ct_fail(CT_EINVAL, "ct_repair_noalloc: null argument");
    if (metric > CT_HAM1_RANDOM) return ct_fail(CT_EINVAL, "ct_repair_noalloc: unknown metric");
    if (metric == CT_TIER_EUCLID && n && !d_pos_q16)
        return ct_fail(CT_EINVAL, "ct_repair_noalloc: TIER_EUCLID needs particle positions");
    if (n > kRows)
        return ct_fail(CT_EINVAL, "ct_repair_noalloc: more rows than the static scratch holds (CT_NOALLOC_MAX_ROWS = " +
                                      std::to_string(kRows) + "); split the call or use ct_repair");
    if (s->n_valid == 0) return ct_fail(CT_EEMPTY, "ct_repair_noalloc: the space has no valid configuration");
    if (s->n_valid > CT_MAX_VALID)
        return ct_fail(CT_EINVAL, "ct_repair_noalloc: more valid configurations than 32-bit positions can name");
    if (n == 0) return CT_OK;
    int dev = -1;
    CT_HIP(hipGetDevice(&dev));
    if (dev != s->device) return ct_fail(CT_EINVAL, "ct_repair_noalloc: the space lives on another device");
    uint8_t* base = nullptr;
    if (int rc = scratch_on_current_device(dev, &base)) return rc;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    RepairSet h{};
    h.S = s->d_dev;
    h.R = s->dev.R;
    h.n_sub = s->dev.n_sub;
    h.rows = d_rows;
    h.n = (uint32_t)n;
    h.metric = metric;
    h.seed = seed;
    h.gen = nullptr;
    h.gen_value = generation;
    h.who = d_who;
    h.pos_q16 = d_pos_q16;
    h.out_rows = d_out_rows;
    h.out_pos = d_out_pos;
    h.apply = nullptr;
    h.list = reinterpret_cast<uint32_t*>(base + kOffList);
    h.list_ins = reinterpret_cast<uint64_t*>(base + kOffListIns);
    h.fb_list = reinterpret_cast<uint32_t*>(base + kOffFbList);
    h.fb_ins = reinterpret_cast<uint64_t*>(base + kOffFbIns);
    h.part_key = reinterpret_cast<uint64_t*>(base + kOffPartKey);
    h.part_pos = reinterpret_cast<uint32_t*>(base + kOffPartPos);
    h.count = reinterpret_cast<uint32_t*>(base + kOffCount);
    h.tally = nullptr;
    uint32_t* prep_off = reinterpret_cast<uint32_t*>(base + kOffPrep);
    RepairSet* d_set = reinterpret_cast<RepairSet*>(base + kOffSet);

    RepairPasses rp;
    uint32_t* w = reinterpret_cast<uint32_t*>(base + kOffPlan);
    rp.plan.cand_off = w;
    rp.plan.item_off = w + 2;
    rp.plan.parts = w + 2 * (1 + kRepairClasses);
    rp.plan.done = rp.plan.parts + 1;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, st, h, d_set, prep_off, rp.plan.done);
    CT_HIP(hipGetLastError());
    rp.n_sets = 1;
    rp.d_sets = d_set;
    rp.d_prep_off = prep_off;
    rp.total_n = (uint32_t)n;
    rp.class_mask = 1u << repair_class(metric, s->R);
    rp.fb_class_mask =
        (metric == CT_TIER_EUCLID || metric == CT_TIER_RANDOM) ? 1u << repair_class(CT_HAMMING, s->R) : 0u;
    rp.euclid_tab = s->dev.max_radix * (s->dev.R < 32 ? s->dev.R + 1 : s->dev.R);
    return launch_repair_passes(rp, true, st);
}
