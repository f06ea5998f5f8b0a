// extern "C" entry points of libct: argument validation, handle ownership,
// device allocation and launch sequencing.  All arithmetic of the method
// runs in the kernels of space.hip, repair.hip and step.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ct_host.h"

namespace {
thread_local std::string g_err = "no error";

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int require_device() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) return ct_fail(CT_EDEVICE, "no HIP device available");
    return CT_OK;
}

// Check a constraint program's stack discipline and operands; returns the largest parameter read (-1: none).
int check_program(const uint32_t* code, uint32_t b, uint32_t e, uint32_t n_params, int* max_param,
                  std::string* why) {
    int depth = 0;
    *max_param = -1;
    for (uint32_t pc = b; pc < e;) {
        uint32_t w = code[pc++];
        uint32_t op = w & 0xFFu;
        int32_t imm = (int32_t)w >> 8;
        switch (op) {
        case OP_PARAM:
            if (imm < 0 || (uint32_t)imm >= n_params) { *why = "parameter id out of range"; return -1; }
            *max_param = std::max(*max_param, imm);
            depth++;
            break;
        case OP_CONST: depth++; break;
        case OP_CONST64:
            if (pc + 2 > e) { *why = "truncated 64-bit constant"; return -1; }
            pc += 2;
            depth++;
            break;
        case OP_NEG: case OP_ABS: case OP_NOT:
            if (depth < 1) { *why = "stack underflow"; return -1; }
            break;
        default:
            if (op < OP_ADD || op > OP_LAST) { *why = "unknown opcode " + std::to_string(op); return -1; }
            if (depth < 2) { *why = "stack underflow"; return -1; }
            depth--;
        }
        if (depth > CT_STACK) { *why = "stack deeper than 16"; return -1; }
    }
    if (depth != 1) { *why = "program must leave exactly one value"; return -1; }
    return 0;
}

// Scan partitionings chosen by the autotuner, by group shape (process-wide).
std::mutex g_tune_mu;
std::map<std::string, RepairTune> g_tune;

// Shape of a group of runs: per run (algorithm, row bytes, parameters, log2 |V|, log2 P, aware or
// not), sorted.
std::string group_shape(const std::vector<ct_pop*>& pops) {
    std::vector<std::string> parts;
    auto lg = [](uint64_t x) { uint32_t k = 0; while (x >>= 1) ++k; return k; };
    for (const ct_pop* p : pops) {
        const PopDev& d = p->dev;
        parts.push_back(std::to_string(d.algo) + "," + std::to_string(d.R) + "," + std::to_string(d.D) + "," +
                        std::to_string(lg(d.n_valid)) + "," + std::to_string(lg(d.P)) + "," + std::to_string(d.unaware));
    }
    std::sort(parts.begin(), parts.end());
    std::string s;
    for (const std::string& x : parts) s += x + ";";
    return s;
}

template <typename T>
int dalloc(ct_pop* p, T** ptr, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return ct_fail(CT_ENOMEM, "hipMalloc failed");
    p->allocs.push_back(q);
    p->dev_bytes += std::max<size_t>(n, 1) * sizeof(T);
    *ptr = reinterpret_cast<T*>(q);
    return CT_OK;
}

}  // namespace

int batch_fill(ct_batch* b, const std::vector<ct_pop*>& pops) {
    if (pops.size() > 4096) return ct_fail(CT_EINVAL, "batch: at most 4096 populations");
    const uint32_t n = (uint32_t)pops.size();
    std::vector<PopDev> pd;
    std::vector<uint32_t> ind_off{0}, ga_off{0}, ff_off{0};
    std::vector<RepairSet> setsA, setsC;
    uint32_t maskA = 0, fbA = 0, max_pop = 0, tabA = 0;
    for (ct_pop* p : pops) {
        const PopDev& d = p->dev;
        pd.push_back(d);
        ind_off.push_back(ind_off.back() + d.P);
        ff_off.push_back(ff_off.back() + (d.algo == CT_FIREFLY ? d.P : 0u));
        RepairSet r{};
        r.S = d.S;
        r.R = d.R;
        r.n_sub = p->space->dev.n_sub;
        r.rows = d.trial;
        r.n = d.P;
        r.metric = d.algo == CT_DE ? CT_INDEX_L1 : d.algo == CT_GA ? CT_TIER_RANDOM : CT_TIER_EUCLID;
        r.seed = d.seed;
        r.gen = d.state;
        r.who = nullptr;
        r.pos_q16 = d.algo == CT_PSO ? d.X : d.algo == CT_FIREFLY ? d.Xn : nullptr;
        r.out_rows = d.out;
        r.out_pos = d.tpos;
        r.apply = nullptr;
        r.list = p->r_list;
        r.list_ins = p->r_list_ins;
        r.fb_list = p->r_fb;
        r.fb_ins = p->r_fb_ins;
        r.count = d.rcount;
        r.part_key = p->r_part_key;
        r.part_pos = p->r_part_pos;
        r.tally = d.tally;
        setsA.push_back(r);
        maskA |= 1u << repair_class(r.metric, d.R);
        if (r.metric == CT_TIER_EUCLID || r.metric == CT_TIER_RANDOM) fbA |= 1u << repair_class(CT_HAMMING, d.R);
        if (r.metric == CT_TIER_EUCLID) tabA = std::max(tabA, p->space->dev.max_radix * (d.R < 32 ? d.R + 1 : d.R));
        if (d.algo == CT_GA) {
            RepairSet m = r;
            m.metric = CT_HAM1_RANDOM;
            m.rows = d.out;
            m.apply = d.apply;
            m.count = d.rcount + 2;
            m.tally = d.tally + 1;
            setsC.push_back(m);
            ga_off.push_back(ga_off.back() + d.P);
        }
        max_pop = std::max(max_pop, d.P);
    }
    // a changed group invalidates any captured graph
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (n > b->cap || !b->d_pops) {
        for (void* q : b->owned) (void)hipFree(q);
        b->owned.clear();
        const uint32_t cap = std::max<uint32_t>(n, 1);
        void* q = nullptr;
        auto own = [&](size_t bytes) -> void* {
            q = nullptr;
            if (hipMalloc(&q, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
            b->owned.push_back(q);
            return q;
        };
        b->d_pops = (PopDev*)own(cap * sizeof(PopDev));
        b->d_ind_off = (uint32_t*)own((cap + 1) * 4);
        b->d_ga_off = (uint32_t*)own((cap + 1) * 4);
        b->d_ff_off = (uint32_t*)own((cap + 1) * 4);
        b->d_setsA = (RepairSet*)own(cap * sizeof(RepairSet));
        b->d_setsC = (RepairSet*)own(cap * sizeof(RepairSet));
        if (!b->d_pops || !b->d_ind_off || !b->d_ga_off || !b->d_ff_off || !b->d_setsA || !b->d_setsC) {
            b->cap = 0;
            b->d_pops = nullptr;
            return ct_fail(CT_ENOMEM, "batch: hipMalloc failed");
        }
        int rc = repair_plan_alloc(b->passA.plan, cap, b->owned);
        if (!rc) rc = repair_plan_alloc(b->passC.plan, cap, b->owned);
        if (rc) {
            b->cap = 0;
            b->d_pops = nullptr;
            return rc;
        }
        b->cap = cap;
    }
    auto upload = [&](void* dst, const void* src, size_t bytes) -> int {
        if (bytes && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return ct_fail(CT_EDEVICE, "batch: descriptor upload failed");
        return CT_OK;
    };
    int rc;
    if ((rc = upload(b->d_pops, pd.data(), pd.size() * sizeof(PopDev))) ||
        (rc = upload(b->d_ind_off, ind_off.data(), ind_off.size() * 4)) ||
        (rc = upload(b->d_setsA, setsA.data(), setsA.size() * sizeof(RepairSet))) ||
        (rc = upload(b->d_setsC, setsC.data(), setsC.size() * sizeof(RepairSet))) ||
        (rc = upload(b->d_ga_off, ga_off.data(), ga_off.size() * 4)) ||
        (rc = upload(b->d_ff_off, ff_off.data(), ff_off.size() * 4)))
        return rc;
    b->pops = pops;
    b->n = n;
    b->total_ind = ind_off.back();
    b->n_ga = (uint32_t)setsC.size();
    b->total_ff = ff_off.back();
    b->max_pop = max_pop;
    // main repair pass: every run (its prep items are its individuals)
    b->passA.fan = &b->fan;
    b->passC.fan = &b->fan;
    b->passA.n_sets = n;
    b->passA.d_sets = b->d_setsA;
    b->passA.d_prep_off = b->d_ind_off;
    b->passA.total_n = b->total_ind;
    b->passA.class_mask = maskA;
    b->passA.fb_class_mask = fbA;
    b->passA.euclid_tab = tabA;
    // GA mutation pass
    b->passC.n_sets = b->n_ga;
    b->passC.d_sets = b->d_setsC;
    b->passC.d_prep_off = b->d_ga_off;
    b->passC.total_n = ga_off.back();
    b->passC.class_mask = 0;
    for (ct_pop* p : pops)
        if (p->dev.algo == CT_GA) b->passC.class_mask |= 1u << repair_class(CT_HAM1_RANDOM, p->dev.R);
    b->passC.fb_class_mask = 0;
    // a group of a shape tuned before reuses that partitioning
    b->shape = group_shape(pops);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(b->shape);
        b->tuned = it != g_tune.end();
        b->tune_cand.clear();
        b->tune_ms.clear();
        b->passA.tune = b->tuned ? it->second : RepairTune{};
        if (!b->tuned) b->passA.tune.mode = kScanFused;
    }
    return CT_OK;
}

int batch_build(const std::vector<ct_pop*>& pops, ct_batch** out, hipStream_t st) {
    (void)st;
    *out = nullptr;
    ct_batch* b = new ct_batch();
    // one run has one scan class per pass: only groups get the auxiliary streams
    int rc = pops.size() > 1 ? fan_create(&b->fan) : CT_OK;
    if (!rc) rc = batch_fill(b, pops);
    if (rc) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return CT_OK;
}

uint64_t pop_footprint_bytes(uint32_t algo, uint32_t P, uint32_t D, uint32_t R, uint64_t n_valid, uint32_t unaware) {
    const uint64_t p = P, pd = (uint64_t)P * D;
    const uint64_t slots = std::max<uint64_t>(P, kRepairMaxItems);
    uint64_t b = 16 + 16 + 16 + 8 + 2 * p * R + 4 * p + p;      // state, tally, rcount, best, trial, out, tpos, apply
    if (algo == CT_PSO) b += pd * (4 + 8 + 4) + 8 * p;           // X, V, PB, f_pb, pb_pos
    else b += 8 * p;                                              // pos, f
    if (algo == CT_FIREFLY) b += pd * (4 + 4);                    // X, Xn
    if (unaware && (algo == CT_DE || algo == CT_GA)) b += p * R + 16 * p;                    // prow, pL, tL
    else if (algo == CT_DE) b += (n_valid + 31) / 32 * 4 + std::max<uint64_t>(n_valid, 1) * 4;   // member, claim
    if (algo == CT_GA) b += 8 * p + 4 * p;                        // beta table, sorted
    b += 4 * p + 8 * p + 4 * p + 8 * p + slots * (8 + 4);         // repair scratch
    return b;
}

uint64_t batch_bytes(uint32_t cap) {
    const uint64_t c = std::max<uint32_t>(cap, 1);
    const uint64_t plan = ((c + 1) * 6 + c) * 4;
    return c * sizeof(PopDev) + 3 * (c + 1) * 4 + 2 * c * sizeof(RepairSet) + 2 * plan;
}

void batch_free(ct_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    for (ct_batch* l : b->lanes) batch_free(l);
    for (hipStream_t q : b->lane_st)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : b->lane_done)
        if (e) (void)hipEventDestroy(e);
    if (b->lane_fork) (void)hipEventDestroy(b->lane_fork);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void* q : b->owned) (void)hipFree(q);
    fan_destroy(&b->fan);
    delete b;
}

int space_prepare(const int64_t* values, const uint32_t* radices, uint32_t n_params, const uint32_t* code,
                  const uint32_t* cons_offsets, uint32_t n_cons, ct_space** out) {
    if (!values || !radices || !out || (n_cons && (!code || !cons_offsets)))
        return ct_fail(CT_EINVAL, "ct_space_build: null argument");
    *out = nullptr;
    if (n_params < 1 || n_params > CT_MAX_PARAMS) return ct_fail(CT_EINVAL, "ct_space_build: 1..32 parameters supported");
    if (n_cons > CT_MAX_PROGRAMS) return ct_fail(CT_EINVAL, "ct_space_build: at most 64 constraint programs");
    unsigned __int128 N = 1;
    uint32_t n_vals = 0, max_radix = 0;
    for (uint32_t j = 0; j < n_params; j++) {
        if (radices[j] < 1 || radices[j] > CT_MAX_RADIX) return ct_fail(CT_EINVAL, "ct_space_build: radix must be 1..255");
        N *= radices[j];
        n_vals += radices[j];
        max_radix = std::max(max_radix, radices[j]);
    }
    if (N >= ((unsigned __int128)1 << CT_MAX_CARTESIAN_LOG2))
        return ct_fail(CT_EINVAL, "ct_space_build: Cartesian size must be below 2^46");
    // validate programs and sort them into prefix-only / the rest
    std::vector<int> maxp(n_cons);
    for (uint32_t c = 0; c < n_cons; c++) {
        if (cons_offsets[c] > cons_offsets[c + 1]) return ct_fail(CT_EINVAL, "ct_space_build: offsets not ascending");
        std::string why;
        if (check_program(code, cons_offsets[c], cons_offsets[c + 1], n_params, &maxp[c], &why))
            return ct_fail(CT_EINVAL, "ct_space_build: program " + std::to_string(c) + ": " + why);
    }
    int rc = require_device();
    if (rc) return rc;

    ct_space* s = new ct_space();
    s->D = n_params;
    s->R = n_params <= 4 ? 4 : n_params <= 8 ? 8 : n_params <= 16 ? 16 : 32;
    s->n_cons = n_cons;
    s->values.assign(values, values + n_vals);
    s->radices.assign(radices, radices + n_params);
    s->n_cartesian = (uint64_t)N;
    (void)hipGetDevice(&s->device);
    DevSpace& S = s->dev;
    S.D = n_params;
    S.R = s->R;
    S.N = (uint64_t)N;
    S.max_radix = max_radix;
    // prefix split: the longest leading run of parameters whose product is at most
    // min(2^24, N / 64), so the prefix table stays small and every prefix owns at least one
    // wave's worth of inner configurations; constraints over the prefix alone are then
    // evaluated once per prefix and invalid prefixes skip their inner configurations
    const uint64_t cap = std::max<uint64_t>(1, std::min<uint64_t>(1ull << 24, (uint64_t)N / 64));
    uint64_t Ps = 1;
    uint32_t split = 0;
    while (split < n_params && Ps * radices[split] <= cap) Ps *= radices[split++];
    // With inner patterns (below) the bitmask of the inner part costs no evaluation per
    // configuration, so the split that needs the fewest evaluations -- one per prefix plus one
    // per (context, inner configuration) -- wins when its patterns fit.
    {
        std::vector<uint32_t> used(n_cons, 0u);
        for (uint32_t c = 0; c < n_cons; c++)
            for (uint32_t pc = cons_offsets[c]; pc < cons_offsets[c + 1];) {
                const uint32_t w = code[pc++];
                if ((w & 0xFFu) == OP_PARAM) used[c] |= 1u << ((int32_t)w >> 8);
                else if ((w & 0xFFu) == OP_CONST64) pc += 2;
            }
        uint64_t best = ~0ull, P = 1;
        for (uint32_t sp = 1; sp < n_params; sp++) {
            P *= radices[sp - 1];
            if (P > (1ull << 24)) break;
            const uint64_t I = (uint64_t)N / P;
            if (I >= (1ull << 31)) continue;
            const uint32_t pre = (uint32_t)((1ull << sp) - 1);
            uint32_t cx = 0;
            for (uint32_t c = 0; c < n_cons; c++)
                if (used[c] & ~pre) cx |= used[c] & pre;
            uint64_t nctx = 1;
            for (uint32_t j = 0; j < sp; j++)
                if (cx & (1u << j)) nctx *= radices[j];
            if (nctx * ((I + 63) / 64 + 1) * 64 > kPatternBits) continue;
            const uint64_t cost = P + nctx * I;
            if (cost < best) { best = cost; split = sp; Ps = P; }
        }
    }
    S.split = split;
    S.P_s = Ps;
    S.I_s = S.N / Ps;
    ct_magic((uint32_t)S.I_s, &S.Is_m, &S.Is_l);
    uint64_t stride = 1;
    uint32_t off = 0;
    for (uint32_t j = 0; j < n_params; j++) S.val_off[j] = 0;
    for (uint32_t j = 0; j < n_params; j++) {
        S.radix[j] = radices[j];
        ct_magic(radices[j], &S.mag_m[j], &S.mag_l[j]);
        S.val_off[j] = off;
        off += radices[j];
    }
    for (uint32_t j = n_params; j-- > 0;) {
        S.stride[j] = stride;
        stride *= radices[j];
    }
    std::vector<uint32_t> order;
    for (uint32_t c = 0; c < n_cons; c++)
        if (maxp[c] < (int)split) order.push_back(c);
    S.n_pre = (uint32_t)order.size();
    for (uint32_t c = 0; c < n_cons; c++)
        if (maxp[c] >= (int)split) order.push_back(c);
    S.n_cons = n_cons;
    std::vector<uint32_t> code2;
    for (uint32_t k = 0; k < n_cons; k++) {
        uint32_t c = order[k];
        S.cons_off[k] = (uint32_t)code2.size();
        code2.insert(code2.end(), code + cons_offsets[c], code + cons_offsets[c + 1]);
    }
    S.cons_off[n_cons] = (uint32_t)code2.size();
    // Scope tables for programs over few parameters (their scope: the parameters they read).
    // Programs of one class (prefix programs [0, n_pre), inner programs [n_pre, n_cons)) join a
    // table of the same class when the union of the scopes stays within CT_TAB_SCOPE parameters
    // and CT_TAB_BITS bits (the smallest such union); the table's first program holds it with
    // the member set, the others are marked covered.  Every tabled program also has its own
    // table (entries [n_cons, 2 n_cons) of the descriptors): those are evaluated first, the
    // shared tables are then their ANDs by lookup.  Table words: own tables, then shared ones.
    s->tab_meta.assign((size_t)std::max<uint32_t>(n_cons, 1) * 2 * CT_TAB_META, 0u);
    s->tab_words = 0;
    auto scope_bits = [&](uint32_t sc) {
        uint64_t b = 1;
        for (uint32_t j = 0; j < n_params; j++)
            if (sc & (1u << j)) b *= radices[j];
        return b;
    };
    auto fill_meta = [&](uint32_t* m, uint32_t scope, uint64_t members) {
        std::vector<uint32_t> sc;
        for (uint32_t j = 0; j < n_params; j++)
            if (scope & (1u << j)) sc.push_back(j);
        const uint64_t bits = scope_bits(scope);
        m[0] = (uint32_t)s->tab_words;
        m[1] = (uint32_t)sc.size();
        m[2] = (uint32_t)bits;
        uint32_t st2 = 1;
        for (size_t q = sc.size(); q-- > 0;) {           // last scope parameter fastest
            m[4 + q] = (st2 << 5) | sc[q];
            const uint32_t j = sc[q];
            m[12 + j / 4] |= (st2 & 0xFFu) << (8 * (j % 4));
            m[20 + j / 4] |= ((st2 >> 8) & 0xFFu) << (8 * (j % 4));
            st2 *= radices[sc[q]];
        }
        m[28] = (uint32_t)members;
        m[29] = (uint32_t)(members >> 32);
        s->tab_words += (bits + 63) / 64;
    };
    struct TabGroup { uint32_t leader, scope; uint64_t members; };
    std::vector<TabGroup> groups;
    for (uint32_t k = 0; k < n_cons; k++) {
        s->tab_meta[(size_t)k * CT_TAB_META] = ~0u;
        s->tab_meta[(size_t)(n_cons + k) * CT_TAB_META] = ~0u;
        uint32_t used = 0;
        for (uint32_t pc = S.cons_off[k]; pc < S.cons_off[k + 1];) {
            const uint32_t w = code2[pc++];
            if ((w & 0xFFu) == OP_PARAM) used |= 1u << ((int32_t)w >> 8);
            else if ((w & 0xFFu) == OP_CONST64) pc += 2;
        }
        if ((uint32_t)__builtin_popcount(used) > CT_TAB_SCOPE || scope_bits(used) > CT_TAB_BITS) continue;
        fill_meta(&s->tab_meta[(size_t)(n_cons + k) * CT_TAB_META], used, 1ull << k);   // its own table
        const bool pre = k < S.n_pre;
        size_t pick = groups.size();
        uint64_t pick_bits = ~0ull;
        for (size_t g = 0; g < groups.size(); g++) {
            if ((groups[g].leader < S.n_pre) != pre) continue;
            const uint32_t u = groups[g].scope | used;
            const uint64_t b = scope_bits(u);
            if ((uint32_t)__builtin_popcount(u) <= CT_TAB_SCOPE && b <= CT_TAB_BITS && b < pick_bits) {
                pick = g;
                pick_bits = b;
            }
        }
        if (pick == groups.size()) {
            groups.push_back(TabGroup{k, used, 1ull << k});
        } else {
            groups[pick].scope |= used;
            groups[pick].members |= 1ull << k;
            s->tab_meta[(size_t)k * CT_TAB_META] = CT_TAB_COVERED;
        }
    }
    s->own_words = s->tab_words;
    for (const TabGroup& g : groups) {
        uint32_t* m = &s->tab_meta[(size_t)g.leader * CT_TAB_META];
        if (__builtin_popcountll(g.members) == 1) {      // alone: its own table
            std::copy(&s->tab_meta[(size_t)(n_cons + g.leader) * CT_TAB_META],
                      &s->tab_meta[(size_t)(n_cons + g.leader + 1) * CT_TAB_META], m);
        } else {
            fill_meta(m, g.scope, g.members);
        }
    }
    // inner patterns: the inner programs read the inner parameters and a few prefix parameters
    // (the context); when every context's pattern over the inner configurations is small, the
    // bitmask of a valid prefix is its context's pattern
    {
        uint32_t used = 0;
        for (uint32_t k = S.n_pre; k < n_cons; k++)
            for (uint32_t pc = S.cons_off[k]; pc < S.cons_off[k + 1];) {
                const uint32_t w = code2[pc++];
                if ((w & 0xFFu) == OP_PARAM) used |= 1u << ((int32_t)w >> 8);
                else if ((w & 0xFFu) == OP_CONST64) pc += 2;
            }
        uint64_t nctx = 1;
        S.n_cx = 0;
        for (uint32_t j = 0; j < split; j++)
            if (used & (1u << j)) { S.cx[S.n_cx++] = j; nctx *= radices[j]; }
        uint64_t st2 = 1;
        for (uint32_t q = S.n_cx; q-- > 0;) {
            const uint32_t j = S.cx[q];
            S.cx[q] = (uint32_t)(st2 << 5) | j;
            st2 *= radices[j];
        }
        s->n_ctx = (split < n_params && nctx * ((S.I_s + 63) / 64 + 1) * 64 <= kPatternBits)
                       ? nctx : 0;
    }
    s->lds_values_bytes = (size_t)n_vals * sizeof(int64_t);
    s->code = std::move(code2);
    *out = s;
    return CT_OK;
}

int space_realize(ct_space* s, hipStream_t st, uint64_t byte_limit) {
    const size_t n_vals = s->values.size();
    if (hipMalloc(&s->d_values, n_vals * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&s->d_code, std::max<size_t>(s->code.size(), 1) * sizeof(uint32_t)) != hipSuccess)
        return ct_fail(CT_ENOMEM, "ct_space_build: hipMalloc failed");
    if (hipMemcpyAsync(s->d_values, s->values.data(), n_vals * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        (s->code.size() && hipMemcpyAsync(s->d_code, s->code.data(), s->code.size() * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, st) != hipSuccess))
        return ct_fail(CT_EDEVICE, "ct_space_build: upload failed");
    s->dev.values = s->d_values;
    s->dev.code = s->d_code;
    if (hipMalloc(&s->d_tab_meta, s->tab_meta.size() * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&s->d_tabs, std::max<uint64_t>(s->tab_words, 1) * sizeof(uint64_t)) != hipSuccess)
        return ct_fail(CT_ENOMEM, "ct_space_build: hipMalloc failed");
    if (hipMemcpyAsync(s->d_tab_meta, s->tab_meta.data(), s->tab_meta.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return ct_fail(CT_EDEVICE, "ct_space_build: upload failed");
    s->dev.tab_meta = s->d_tab_meta;
    s->dev.tabs = s->d_tabs;
    s->byte_limit = byte_limit;
    int rc = space_build_device(s, st);
    if (rc) return rc;
    if (hipMalloc(&s->d_dev, sizeof(DevSpace)) != hipSuccess) return ct_fail(CT_ENOMEM, "ct_space_build: hipMalloc failed");
    if (hipMemcpy(s->d_dev, &s->dev, sizeof(DevSpace), hipMemcpyHostToDevice) != hipSuccess)
        return ct_fail(CT_EDEVICE, "ct_space_build: upload failed");
    s->dev_bytes = space_resident_bytes(s, s->n_valid);
    return CT_OK;
}


int ct_fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

extern "C" {

const char* ct_last_error(void) { return g_err.c_str(); }

int ct_version(void) { return 2; }

int ct_space_build(const int64_t* values, const uint32_t* radices, uint32_t n_params, const uint32_t* code,
                   const uint32_t* cons_offsets, uint32_t n_cons, void* stream, ct_space** out) {
    if (!out) return ct_fail(CT_EINVAL, "ct_space_build: null argument");
    *out = nullptr;
    ct_space* s = nullptr;
    int rc = space_prepare(values, radices, n_params, code, cons_offsets, n_cons, &s);
    if (rc) return rc;
    rc = space_realize(s, as_stream(stream), 0);
    if (rc) {
        ct_space_free(s);
        return rc;
    }
    *out = s;
    return CT_OK;
}

int ct_space_count(const ct_space* s, uint64_t* n_valid, uint64_t* n_cartesian) {
    if (!s) return ct_fail(CT_EINVAL, "ct_space_count: null space");
    if (n_valid) *n_valid = s->n_valid;
    if (n_cartesian) *n_cartesian = s->n_cartesian;
    return CT_OK;
}

int ct_space_info(const ct_space* s, uint32_t* n_params, uint32_t* row_bytes) {
    if (!s) return ct_fail(CT_EINVAL, "ct_space_info: null space");
    if (n_params) *n_params = s->D;
    if (row_bytes) *row_bytes = s->R;
    return CT_OK;
}

int ct_space_valid_list(const ct_space* s, const uint64_t** d_lin, const uint8_t** d_rows) {
    if (!s) return ct_fail(CT_EINVAL, "ct_space_valid_list: null space");
    if (d_lin) *d_lin = s->d_lin;
    if (d_rows) *d_rows = s->d_rows;
    return CT_OK;
}

int ct_space_bitmask(const ct_space* s, const uint64_t** d_words, uint64_t* n_words) {
    if (!s) return ct_fail(CT_EINVAL, "ct_space_bitmask: null space");
    if (d_words) *d_words = s->d_words;
    if (n_words) *n_words = s->n_words;
    return CT_OK;
}

int ct_space_copy_list(const ct_space* s, uint64_t* d_lin, uint8_t* d_rows, void* stream) {
    if (!s) return ct_fail(CT_EINVAL, "ct_space_copy_list: null space");
    hipStream_t st = as_stream(stream);
    if (s->n_valid && d_lin)
        CT_HIP(hipMemcpyAsync(d_lin, s->d_lin, s->n_valid * 8, hipMemcpyDeviceToDevice, st));
    if (s->n_valid && d_rows)
        CT_HIP(hipMemcpyAsync(d_rows, s->d_rows, s->n_valid * s->R, hipMemcpyDeviceToDevice, st));
    return CT_OK;
}

int ct_space_copy_bitmask(const ct_space* s, uint64_t* d_words, void* stream) {
    if (!s || !d_words) return ct_fail(CT_EINVAL, "ct_space_copy_bitmask: null argument");
    CT_HIP(hipMemcpyAsync(d_words, s->d_words, s->n_words * 8, hipMemcpyDeviceToDevice, as_stream(stream)));
    return CT_OK;
}

void ct_space_free(ct_space* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    void* bufs[] = {s->d_values, s->d_code, s->d_prefix, s->d_words, s->d_lin, s->d_rows, s->d_prevnext,
                    s->d_grp_off, s->d_dir8, s->d_boxes, s->d_dev, s->d_tab_meta, s->d_tabs};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete s;
}

int ct_valid_mask(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint8_t* d_out, void* stream) {
    if (!s || (n && (!d_rows || !d_out))) return ct_fail(CT_EINVAL, "ct_valid_mask: null argument");
    return launch_valid_mask(s, d_rows, n, d_out, as_stream(stream));
}

int ct_rank(const ct_space* s, const uint8_t* d_rows, uint64_t n, int64_t* d_pos, void* stream) {
    if (!s || (n && (!d_rows || !d_pos))) return ct_fail(CT_EINVAL, "ct_rank: null argument");
    return launch_rank(s, d_rows, n, d_pos, as_stream(stream));
}

// ct_repair, and with `enumerate` ct_repair_enum: shells through the bitmask first, the scans for
// what they leave
static int repair_call(const char* name, const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric,
                       uint64_t seed, uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16,
                       uint8_t* d_out_rows, uint32_t* d_out_pos, void* stream, bool enumerate, uint64_t max_lookups,
                       uint64_t* h_stats) {
    const std::string nm(name);
    if (!s || (n && (!d_rows || !d_out_rows || !d_out_pos))) return ct_fail(CT_EINVAL, nm + ": null argument");
    if (metric > CT_HAM1_RANDOM) return ct_fail(CT_EINVAL, nm + ": unknown metric");
    if (metric == CT_TIER_EUCLID && n && !d_pos_q16)
        return ct_fail(CT_EINVAL, nm + ": TIER_EUCLID needs particle positions");
    if (n > 0x7FFFFFFFull) return ct_fail(CT_EINVAL, nm + ": at most 2^31-1 rows per call");
    if (s->n_valid == 0) return ct_fail(CT_EEMPTY, nm + ": the space has no valid configuration");
    if (s->n_valid > CT_MAX_VALID)
        return ct_fail(CT_EINVAL, nm + ": more valid configurations than 32-bit positions can name");
    if (h_stats) h_stats[0] = h_stats[1] = 0;
    if (n == 0) return CT_OK;
    hipStream_t st = as_stream(stream);
    // one candidate set: scratch lists, per-part winners, the set itself and its plan (enumeration:
    // a second list, counters, descriptor and the statistics)
    const uint64_t slots = std::max<uint64_t>(n, kRepairTargetWaves);
    const size_t bytes = n * (4 + 8 + 4 + 8) + slots * (8 + 4) + 4 * 4 + 2 * 4 + sizeof(RepairSet) + 64 +
                         (enumerate ? n * (4 + 8) + sizeof(RepairSet) + 16 + 64 : 0);
    uint8_t* buf = nullptr;
    CT_HIP(hipMallocAsync((void**)&buf, bytes, st));
    RepairSet h{};
    size_t o = 0;
    auto take = [&](size_t sz) { void* q = buf + o; o += (sz + 7) & ~size_t(7); return q; };
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
    h.list = (uint32_t*)take(n * 4);
    h.list_ins = (uint64_t*)take(n * 8);
    h.fb_list = (uint32_t*)take(n * 4);
    h.fb_ins = (uint64_t*)take(n * 8);
    h.part_key = (uint64_t*)take(slots * 8);
    h.part_pos = (uint32_t*)take(slots * 4);
    h.count = (uint32_t*)take(4 * 4);
    h.tally = nullptr;
    uint32_t* prep_off = (uint32_t*)take(2 * 4);
    RepairSet* d_set = (RepairSet*)take(sizeof(RepairSet));
    const uint32_t h_off[2] = {0, (uint32_t)n};
    std::vector<void*> owned;
    RepairPasses rp;
    int rc = repair_plan_alloc(rp.plan, 1, owned);
    if (!rc) {
        CT_HIP(hipMemcpyAsync(d_set, &h, sizeof(RepairSet), hipMemcpyHostToDevice, st));
        CT_HIP(hipMemcpyAsync(prep_off, h_off, sizeof(h_off), hipMemcpyHostToDevice, st));
        rp.n_sets = 1;
        rp.d_sets = d_set;
        rp.d_prep_off = prep_off;
        rp.total_n = (uint32_t)n;
        rp.class_mask = 1u << repair_class(metric, s->R);
        rp.fb_class_mask = (metric == CT_TIER_EUCLID || metric == CT_TIER_RANDOM) ? 1u << repair_class(CT_HAMMING, s->R) : 0u;
        rp.euclid_tab = s->dev.max_radix * (s->dev.R < 32 ? s->dev.R + 1 : s->dev.R);
        if (!enumerate) {
            rc = launch_repair_passes(rp, true, st);
        } else {
            // the candidates enumeration leaves: their own list and counters, same outputs
            RepairSet h2 = h;
            h2.list = (uint32_t*)take(n * 4);
            h2.list_ins = (uint64_t*)take(n * 8);
            h2.count = h.count + 2;
            RepairSet* d_set2 = (RepairSet*)take(sizeof(RepairSet));
            unsigned long long* d_stats = (unsigned long long*)take(16);
            CT_HIP(hipMemcpyAsync(d_set2, &h2, sizeof(RepairSet), hipMemcpyHostToDevice, st));
            RepairPasses rest = rp;
            rest.d_sets = d_set2;
            rc = repair_plan_alloc(rest.plan, 1, owned);
            if (!rc) rc = launch_repair_enum(rp, rest, max_lookups, d_stats, st);
            if (!rc && h_stats) {
                unsigned long long t[2];
                if (hipMemcpyAsync(t, d_stats, sizeof(t), hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    rc = ct_fail(CT_EDEVICE, nm + ": statistics copy failed");
                h_stats[0] = t[0];
                h_stats[1] = t[1];
            }
        }
    }
    (void)hipFreeAsync(buf, st);
    (void)hipStreamSynchronize(st);
    for (void* q : owned) (void)hipFree(q);
    return rc;
}

int ct_repair(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric, uint64_t seed,
              uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16, uint8_t* d_out_rows,
              uint32_t* d_out_pos, void* stream) {
    return repair_call("ct_repair", s, d_rows, n, metric, seed, generation, d_who, d_pos_q16, d_out_rows, d_out_pos,
                       stream, false, 0, nullptr);
}

int ct_repair_enum(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric, uint64_t seed,
                   uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16, uint64_t max_lookups,
                   uint8_t* d_out_rows, uint32_t* d_out_pos, uint64_t* h_stats, void* stream) {
    return repair_call("ct_repair_enum", s, d_rows, n, metric, seed, generation, d_who, d_pos_q16, d_out_rows,
                       d_out_pos, stream, true, max_lookups, h_stats);
}

int ct_pop_create(const ct_space* s, const ct_pop_params* prm, const float* d_objective, void* stream,
                  ct_pop** out) {
    if (!s || !prm || !d_objective || !out) return ct_fail(CT_EINVAL, "ct_pop_create: null argument");
    *out = nullptr;
    const ct_pop_params& q = *prm;
    if (q.algo > CT_FIREFLY) return ct_fail(CT_EINVAL, "ct_pop_create: unknown algorithm");
    if (s->n_valid == 0) return ct_fail(CT_EEMPTY, "ct_pop_create: the space has no valid configuration");
    if (s->n_valid > CT_MAX_VALID)
        return ct_fail(CT_EINVAL, "ct_pop_create: more valid configurations than 32-bit positions can name");
    if (q.pop_size < 1 || q.pop_size > CT_MAX_POP) return ct_fail(CT_EINVAL, "ct_pop_create: pop_size out of range");
    if (q.unaware > 1) return ct_fail(CT_EINVAL, "ct_pop_create: unaware is 0 or 1");
    if (!q.unaware && q.pop_size > s->n_valid)
        return ct_fail(CT_EINVAL, "ct_pop_create: pop_size exceeds the number of valid configurations");
    if (q.algo == CT_DE && q.pop_size < 4) return ct_fail(CT_EINVAL, "ct_pop_create: DE needs pop_size >= 4");
    if (q.unaware && q.algo == CT_DE && q.pop_size > CT_UNAWARE_DE_MAX_POP)
        return ct_fail(CT_EINVAL, "ct_pop_create: the non-aware DE supports pop_size <= 8192");
    if (q.algo == CT_DE && (q.de_method > CT_DE_RANDTOBEST1 || q.de_crossover > CT_DE_EXP))
        return ct_fail(CT_EINVAL, "ct_pop_create: unknown DE operator or crossover");
    if (q.algo == CT_DE && (q.de_method == CT_DE_RAND2 || q.de_method == CT_DE_BEST2) && q.pop_size < 6)
        return ct_fail(CT_EINVAL, "ct_pop_create: the two-difference DE operators need pop_size >= 6");
    if (q.algo == CT_GA && q.ga_crossover > CT_GA_DISRUPTIVE_UNIFORM)
        return ct_fail(CT_EINVAL, "ct_pop_create: unknown GA crossover");
    if (q.algo == CT_DE && q.CR_q32 > (1ull << 32)) return ct_fail(CT_EINVAL, "ct_pop_create: CR_q32 above 2^32");
    if (q.algo == CT_PSO && (q.w_q16 >= 65536 || q.c1_q16 > (1u << 20) || q.c2_q16 > (1u << 20)))
        return ct_fail(CT_EINVAL, "ct_pop_create: PSO coefficients out of range");
    if (q.algo == CT_GA && (q.mutation_chance < 1 || q.beta_b < 1 || q.beta_b > 5 || q.pop_size > 8192))
        return ct_fail(CT_EINVAL, "ct_pop_create: GA needs mutation_chance >= 1, 1 <= beta_b <= 5, pop_size <= 8192");
    if (q.algo == CT_FIREFLY && (q.ff_B0_q16 > (1u << 20) || q.ff_gamma_q16 > (1u << 20) || q.ff_alpha_q16 > (1u << 20)))
        return ct_fail(CT_EINVAL, "ct_pop_create: Firefly B0, gamma and alpha must be at most 2^20 (16.0)");
    for (uint32_t w : q.reserved)
        if (w) return ct_fail(CT_EINVAL, "ct_pop_create: reserved parameter words must be 0");
    int rc = require_device();
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    ct_pop* p = new ct_pop();
    p->space = s;
    p->prm = q;
    PopDev& d = p->dev;
    d.S = s->d_dev;
    d.n_valid = s->n_valid;
    d.algo = q.algo;
    d.P = q.pop_size;
    d.D = s->D;
    d.R = s->R;
    d.seed = q.seed;
    d.F_q16 = q.F_q16;
    d.de_method = q.de_method;
    d.de_cross = q.de_crossover;
    d.ga_cross = q.ga_crossover;
    d.unaware = q.unaware;
    d.CR_q32 = q.CR_q32;
    d.w_q16 = q.w_q16;
    d.c1_q16 = q.c1_q16;
    d.c2_q16 = q.c2_q16;
    d.mut_thresh = q.algo == CT_GA ? (1ull << 32) / q.mutation_chance : 0;   // chance 1: 2^32, every child
    d.M = s->dev.max_radix;
    d.ff_B0 = q.ff_B0_q16;
    d.ff_gamma = q.ff_gamma_q16;
    d.ff_alpha = q.ff_alpha_q16;
    d.obj = d_objective;
    const uint32_t P = d.P;
    auto fail = [&](int code_) {
        ct_pop_free(p);
        return code_;
    };
    const uint64_t slots = std::max<uint64_t>(P, kRepairMaxItems);
    if ((rc = dalloc(p, &d.state, 4)) || (rc = dalloc(p, &d.tally, 2)) || (rc = dalloc(p, &d.rcount, 4)) || (rc = dalloc(p, &d.best, 1)) || (rc = dalloc(p, &d.trial, (size_t)P * d.R)) ||
        (rc = dalloc(p, &d.out, (size_t)P * d.R)) || (rc = dalloc(p, &d.tpos, P)) || (rc = dalloc(p, &d.apply, P)))
        return fail(rc);
    if (q.algo == CT_PSO) {
        if ((rc = dalloc(p, &d.X, (size_t)P * d.D)) || (rc = dalloc(p, &d.V, (size_t)P * d.D)) ||
            (rc = dalloc(p, &d.PB, (size_t)P * d.D)) || (rc = dalloc(p, &d.f_pb, P)) || (rc = dalloc(p, &d.pb_pos, P)))
            return fail(rc);
    } else {
        if ((rc = dalloc(p, &d.pos, P)) || (rc = dalloc(p, &d.f, P))) return fail(rc);
    }
    if (q.algo == CT_FIREFLY) {
        if ((rc = dalloc(p, &d.X, (size_t)P * d.D)) || (rc = dalloc(p, &d.Xn, (size_t)P * d.D))) return fail(rc);
    }
    if (q.unaware && (q.algo == CT_DE || q.algo == CT_GA)) {
        if ((rc = dalloc(p, &d.prow, (size_t)P * d.R)) || (rc = dalloc(p, &d.pL, P)) || (rc = dalloc(p, &d.tL, P)))
            return fail(rc);
    }
    if (q.algo == CT_DE && !q.unaware) {
        size_t words = (s->n_valid + 31) / 32;
        if ((rc = dalloc(p, &d.member, words)) || (rc = dalloc(p, &d.claim, s->n_valid))) return fail(rc);
        if (hipMemsetAsync(d.member, 0, words * 4, st) != hipSuccess ||
            hipMemsetAsync(d.claim, 0xFF, s->n_valid * 4, st) != hipSuccess)
            return fail(ct_fail(CT_EDEVICE, "ct_pop_create: memset failed"));
    }
    if (q.algo == CT_GA) {
        // cumulative Beta(1, b) rank-selection thresholds: floor((P^b - (P-r-1)^b) * 2^32 / P^b)
        std::vector<uint64_t> t(P);
        unsigned __int128 Pb = 1;
        for (uint32_t k = 0; k < q.beta_b; k++) Pb *= P;
        for (uint32_t r = 0; r < P; r++) {
            unsigned __int128 x = 1;
            for (uint32_t k = 0; k < q.beta_b; k++) x *= (P - r - 1);
            t[r] = (uint64_t)(((Pb - x) << 32) / Pb);
        }
        uint64_t* d_beta = nullptr;
        if ((rc = dalloc(p, &d_beta, P)) || (rc = dalloc(p, &d.sorted, P))) return fail(rc);
        if (hipMemcpy(d_beta, t.data(), P * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess)
            return fail(ct_fail(CT_EDEVICE, "ct_pop_create: upload failed"));
        d.beta = d_beta;
    }
    if (hipMemsetAsync(d.tally, 0, 2 * sizeof(unsigned long long), st) != hipSuccess)
        return fail(ct_fail(CT_EDEVICE, "ct_pop_create: memset failed"));
    if ((rc = dalloc(p, &p->r_list, P)) || (rc = dalloc(p, &p->r_list_ins, P)) || (rc = dalloc(p, &p->r_fb, P)) ||
        (rc = dalloc(p, &p->r_fb_ins, P)) || (rc = dalloc(p, &p->r_part_key, slots)) ||
        (rc = dalloc(p, &p->r_part_pos, slots)))
        return fail(rc);
    if ((rc = pop_init_device(p, st))) return fail(rc);
    *out = p;
    return CT_OK;
}

int ct_step(ct_pop* const* pops, uint32_t n_pops, uint32_t n_generations, uint32_t flags, void* stream) {
    if (n_pops && !pops) return ct_fail(CT_EINVAL, "ct_step: null population list");
    if (flags > CT_STEP_GRAPH) return ct_fail(CT_EINVAL, "ct_step: unknown flags");
    for (uint32_t k = 0; k < n_pops; k++)
        if (!pops[k]) return ct_fail(CT_EINVAL, "ct_step: null population");
    hipStream_t st = as_stream(stream);
    if (flags == CT_STEP_PLAIN) {
        for (uint32_t k = 0; k < n_pops; k++)
            if (!pops[k]->single) {
                int rc = batch_build(std::vector<ct_pop*>{pops[k]}, &pops[k]->single, st);
                if (rc) return rc;
            }
        for (uint32_t g = 0; g < n_generations; g++)
            for (uint32_t k = 0; k < n_pops; k++) {
                int rc = batch_generation(pops[k]->single, st);
                if (rc) return rc;
            }
        return CT_OK;
    }
    ct_batch* b = nullptr;
    int rc = ct_batch_create(pops, n_pops, &b);
    if (rc) return rc;
    rc = ct_batch_step(b, n_generations, flags, stream);
    (void)hipStreamSynchronize(st);
    ct_batch_free(b);
    return rc;
}

int ct_batch_create(ct_pop* const* pops, uint32_t n_pops, ct_batch** out) {
    return ct_batch_create_lanes(pops, n_pops, n_pops >= kLaneMinRuns ? kLanes : 1u, out);
}

int ct_batch_create_lanes(ct_pop* const* pops, uint32_t n_pops, uint32_t n_lanes, ct_batch** out) {
    if (!out || (n_pops && !pops)) return ct_fail(CT_EINVAL, "ct_batch_create: null argument");
    if (n_lanes < 1 || n_lanes > kMaxLanes) return ct_fail(CT_EINVAL, "ct_batch_create_lanes: lanes in [1, 8]");
    *out = nullptr;
    std::vector<ct_pop*> v(pops, pops + n_pops);
    for (ct_pop* p : v)
        if (!p) return ct_fail(CT_EINVAL, "ct_batch_create: null population");
    for (size_t a = 0; a < v.size(); a++)
        for (size_t b = a + 1; b < v.size(); b++)
            if (v[a] == v[b]) return ct_fail(CT_EINVAL, "ct_batch_create: a population appears twice");
    n_lanes = std::min<uint32_t>(n_lanes, std::max<uint32_t>((uint32_t)v.size(), 1u));
    if (n_lanes == 1) return batch_build(v, out, nullptr);
    // lanes: sub-batches on streams of their own, forked from and joined back into the caller's
    ct_batch* b = new ct_batch();
    b->pops = v;
    b->n = (uint32_t)v.size();
    int rc = CT_OK;
    // the fork and join events order work of one device: a device-scope release is enough
    const unsigned ev_flags = hipEventDisableTiming | hipEventReleaseToDevice;
    if (hipEventCreateWithFlags(&b->lane_fork, ev_flags) != hipSuccess) rc = ct_fail(CT_EDEVICE, "hipEventCreate failed");
    // the lanes' streams first, one after the other: HIP spreads streams over the device's hardware
    // queues in the order they are created, and two lanes sharing one queue would not overlap
    for (uint32_t l = 0; l < n_lanes && !rc; ++l) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
            rc = ct_fail(CT_EDEVICE, "hipStreamCreate failed");
            break;
        }
        b->lane_st.push_back(q);
        if (hipEventCreateWithFlags(&e, ev_flags) != hipSuccess) {
            rc = ct_fail(CT_EDEVICE, "hipEventCreate failed");
            break;
        }
        b->lane_done.push_back(e);
    }
    for (uint32_t l = 0; l < n_lanes && !rc; ++l) {
        std::vector<ct_pop*> part;
        for (size_t i = l; i < v.size(); i += n_lanes) part.push_back(v[i]);
        ct_batch* lb = nullptr;
        rc = batch_build(part, &lb, nullptr);
        if (!rc) b->lanes.push_back(lb);
    }
    if (rc) {
        batch_free(b);
        return rc;
    }
    b->shape = b->lanes[0]->shape;
    *out = b;
    return CT_OK;
}

namespace {

int batch_step_one(ct_batch* b, uint32_t n_generations, uint32_t flags, hipStream_t st);

// Every lane steps from the state `st` has reached, each on its own stream; `st` then waits for
// all of them.
int step_lanes(ct_batch* b, uint32_t n_generations, uint32_t flags, hipStream_t st) {
    CT_HIP(hipEventRecord(b->lane_fork, st));
    int rc = CT_OK;
    for (size_t l = 0; l < b->lanes.size(); ++l) {
        CT_HIP(hipStreamWaitEvent(b->lane_st[l], b->lane_fork, 0));
        if (!rc) rc = batch_step_one(b->lanes[l], n_generations, flags, b->lane_st[l]);
        CT_HIP(hipEventRecord(b->lane_done[l], b->lane_st[l]));
        CT_HIP(hipStreamWaitEvent(st, b->lane_done[l], 0));
    }
    return rc;
}

}  // namespace

int ct_batch_step(ct_batch* b, uint32_t n_generations, uint32_t flags, void* stream) {
    if (!b) return ct_fail(CT_EINVAL, "ct_batch_step: null batch");
    if (flags != CT_STEP_BATCHED && flags != CT_STEP_GRAPH) return ct_fail(CT_EINVAL, "ct_batch_step: flags");
    hipStream_t st = as_stream(stream);
    if (!b->lanes.empty()) return step_lanes(b, n_generations, flags, st);
    return batch_step_one(b, n_generations, flags, st);
}

namespace {

int batch_step_one(ct_batch* b, uint32_t n_generations, uint32_t flags, hipStream_t st) {
    if (flags == CT_STEP_BATCHED) {
        for (uint32_t g = 0; g < n_generations; g++) {
            int rc = batch_generation(b, st);
            if (rc) return rc;
        }
        return CT_OK;
    }
    if (!b->exec) {
        // capture one generation once; replays need no host work (the generation counter is on the device)
        hipStream_t cs = nullptr;
        CT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        prof_suspend(true);
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? batch_generation(b, cs) : ct_fail(CT_EDEVICE, "hipStreamBeginCapture failed");
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        prof_suspend(false);
        (void)hipStreamDestroy(cs);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e2 != hipSuccess || !g) return ct_fail(CT_EDEVICE, "hipStreamEndCapture failed");
        b->graph = g;
        CT_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    for (uint32_t g = 0; g < n_generations; g++) CT_HIP(hipGraphLaunch(b->exec, st));
    return CT_OK;
}

}  // namespace

int ct_batch_autotune(ct_batch* b, uint32_t n_generations, uint32_t sample_every, uint32_t force, void* stream) {
    if (!b) return ct_fail(CT_EINVAL, "ct_batch_autotune: null batch");
    hipStream_t st = as_stream(stream);
    if (!b->lanes.empty()) {
        // each lane tuned on its own, one after the other on the caller's stream
        for (ct_batch* l : b->lanes)
            if (int rc = ct_batch_autotune(l, n_generations, sample_every, force, stream)) return rc;
        b->tuned = true;
        return CT_OK;
    }
    if (b->tuned && !force) {
        for (uint32_t g = 0; g < n_generations; g++) {
            int rc = batch_generation(b, st);
            if (rc) return rc;
        }
        return CT_OK;
    }
    if (n_generations == 0) return CT_OK;
    if (int rc = batch_autotune(b, n_generations, sample_every, st)) return rc;
    b->tuned = true;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[b->shape] = b->passA.tune;
    }
    // a captured generation holds the old partitioning
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    return CT_OK;
}

int ct_batch_set_tuning(ct_batch* b, uint32_t items, uint32_t min_boxes, uint32_t grid_waves, uint32_t mode) {
    if (!b) return ct_fail(CT_EINVAL, "ct_batch_set_tuning: null batch");
    // items <= kRepairMaxItems keeps every set's (candidate, part) winners within its slots
    if (items < 64 || items > kRepairMaxItems || min_boxes < 1 || min_boxes > (1u << 20) || grid_waves < 64 ||
        grid_waves > (1u << 20) || mode > CT_SCAN_FUSED)
        return ct_fail(CT_EINVAL, "ct_batch_set_tuning: items in [64, 32768], min_boxes in [1, 2^20], "
                                  "grid_waves in [64, 2^20], mode CT_SCAN_SERIAL, _STREAMS or _FUSED");
    for (ct_batch* l : b->lanes)
        if (int rc = ct_batch_set_tuning(l, items, min_boxes, grid_waves, mode)) return rc;
    b->passA.tune = RepairTune{items, min_boxes, grid_waves, mode};
    b->tuned = true;
    b->tune_cand.clear();
    b->tune_ms.clear();
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    return CT_OK;
}

int ct_batch_tuning(const ct_batch* b, uint32_t* items, uint32_t* min_boxes, uint32_t* grid_waves,
                    uint32_t* mode, uint32_t* tuned) {
    if (!b) return ct_fail(CT_EINVAL, "ct_batch_tuning: null batch");
    if (!b->lanes.empty()) {
        const int rc = ct_batch_tuning(b->lanes[0], items, min_boxes, grid_waves, mode, nullptr);
        if (tuned) *tuned = b->tuned ? 1u : 0u;
        return rc;
    }
    if (items) *items = b->passA.tune.items;
    if (min_boxes) *min_boxes = b->passA.tune.min_sub;
    if (grid_waves) *grid_waves = b->passA.tune.grid_waves;
    if (mode) *mode = b->passA.tune.mode;
    if (tuned) *tuned = b->tuned ? 1u : 0u;
    return CT_OK;
}

void ct_batch_free(ct_batch* b) { batch_free(b); }

int ct_pop_read(const ct_pop* p, uint32_t* h_pos, float* h_f, uint32_t* best_pos, float* best_f,
                uint32_t* generation, uint32_t* reinits) {
    if (!p) return ct_fail(CT_EINVAL, "ct_pop_read: null population");
    const PopDev& d = p->dev;
    CT_HIP(hipDeviceSynchronize());
    if (h_pos) CT_HIP(hipMemcpy(h_pos, d.algo == CT_PSO ? d.pb_pos : d.pos, d.P * 4, hipMemcpyDeviceToHost));
    if (h_f) CT_HIP(hipMemcpy(h_f, d.algo == CT_PSO ? d.f_pb : d.f, d.P * 4, hipMemcpyDeviceToHost));
    uint64_t b = 0;
    uint32_t stt[4];
    CT_HIP(hipMemcpy(&b, d.best, 8, hipMemcpyDeviceToHost));
    CT_HIP(hipMemcpy(stt, d.state, 16, hipMemcpyDeviceToHost));
    if (best_pos) *best_pos = (uint32_t)b;
    if (best_f) {
        uint32_t o = (uint32_t)(b >> 32);
        uint32_t bits = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
        memcpy(best_f, &bits, 4);
    }
    if (generation) *generation = stt[0];
    if (reinits) *reinits = stt[1];
    return CT_OK;
}

int ct_pop_evaluated(const ct_pop* p, uint32_t* h_pos) {
    if (!p || !h_pos) return ct_fail(CT_EINVAL, "ct_pop_evaluated: null argument");
    CT_HIP(hipDeviceSynchronize());
    CT_HIP(hipMemcpy(h_pos, p->dev.tpos, p->dev.P * 4, hipMemcpyDeviceToHost));
    return CT_OK;
}

int ct_pop_counters(const ct_pop* p, uint64_t* repairs, uint64_t* mutations) {
    if (!p) return ct_fail(CT_EINVAL, "ct_pop_counters: null population");
    unsigned long long t[2];
    CT_HIP(hipDeviceSynchronize());
    CT_HIP(hipMemcpy(t, p->dev.tally, sizeof(t), hipMemcpyDeviceToHost));
    if (repairs) *repairs = t[0];
    if (mutations) *mutations = t[1];
    return CT_OK;
}

static bool has_rows(const PopDev& d) { return d.unaware && (d.algo == CT_DE || d.algo == CT_GA); }
static uint32_t snapshot_magic(const PopDev& d) { return d.unaware ? 0x43545531u : 0x43545031u; }

static size_t snapshot_size(const PopDev& d) {
    size_t n = 32;
    if (d.algo == CT_PSO) n += (size_t)d.P * d.D * (4 + 8 + 4) + (size_t)d.P * 8 + 4;
    else n += (size_t)d.P * 8;
    if (d.algo == CT_FIREFLY) n += (size_t)d.P * d.D * 4;
    if (has_rows(d)) n += (size_t)d.P * d.D;
    return n;
}

int ct_pop_snapshot(const ct_pop* p, void* h_buf, size_t* len) {
    if (!p || !len) return ct_fail(CT_EINVAL, "ct_pop_snapshot: null argument");
    const PopDev& d = p->dev;
    size_t need = snapshot_size(d);
    if (!h_buf) { *len = need; return CT_OK; }
    if (*len < need) return ct_fail(CT_EINVAL, "ct_pop_snapshot: buffer too small");
    CT_HIP(hipDeviceSynchronize());
    uint8_t* o = static_cast<uint8_t*>(h_buf);
    uint32_t stt[4];
    uint64_t b;
    CT_HIP(hipMemcpy(stt, d.state, 16, hipMemcpyDeviceToHost));
    CT_HIP(hipMemcpy(&b, d.best, 8, hipMemcpyDeviceToHost));
    uint32_t h[8] = {snapshot_magic(d), d.algo, d.P, d.D, stt[0], stt[1], (uint32_t)b, (uint32_t)(b >> 32)};
    memcpy(o, h, 32);
    o += 32;
    if (d.algo == CT_PSO) {
        size_t PD = (size_t)d.P * d.D;
        CT_HIP(hipMemcpy(o, d.X, PD * 4, hipMemcpyDeviceToHost)); o += PD * 4;
        CT_HIP(hipMemcpy(o, d.V, PD * 8, hipMemcpyDeviceToHost)); o += PD * 8;
        CT_HIP(hipMemcpy(o, d.PB, PD * 4, hipMemcpyDeviceToHost)); o += PD * 4;
        CT_HIP(hipMemcpy(o, d.f_pb, d.P * 4, hipMemcpyDeviceToHost)); o += d.P * 4;
        CT_HIP(hipMemcpy(o, d.pb_pos, d.P * 4, hipMemcpyDeviceToHost)); o += d.P * 4;
        memcpy(o, &stt[2], 4);
    } else {
        CT_HIP(hipMemcpy(o, d.pos, d.P * 4, hipMemcpyDeviceToHost)); o += d.P * 4;
        CT_HIP(hipMemcpy(o, d.f, d.P * 4, hipMemcpyDeviceToHost)); o += d.P * 4;
        if (d.algo == CT_FIREFLY) CT_HIP(hipMemcpy(o, d.X, (size_t)d.P * d.D * 4, hipMemcpyDeviceToHost));
        if (has_rows(d)) {
            // member rows, D digits each (the device rows are padded to R bytes)
            std::vector<uint8_t> rows((size_t)d.P * d.R);
            CT_HIP(hipMemcpy(rows.data(), d.prow, rows.size(), hipMemcpyDeviceToHost));
            for (uint32_t i = 0; i < d.P; ++i) memcpy(o + (size_t)i * d.D, rows.data() + (size_t)i * d.R, d.D);
        }
    }
    *len = need;
    return CT_OK;
}

int ct_pop_restore(ct_pop* p, const void* h_buf, size_t len) {
    if (!p || !h_buf) return ct_fail(CT_EINVAL, "ct_pop_restore: null argument");
    PopDev& d = p->dev;
    if (len != snapshot_size(d)) return ct_fail(CT_EINVAL, "ct_pop_restore: size mismatch");
    const uint8_t* o = static_cast<const uint8_t*>(h_buf);
    uint32_t h[8];
    memcpy(h, o, 32);
    o += 32;
    if (h[0] != snapshot_magic(d) || h[1] != d.algo || h[2] != d.P || h[3] != d.D)
        return ct_fail(CT_EINVAL, "ct_pop_restore: snapshot is for a different run shape");
    // every field is checked before anything reaches the device, so a rejected snapshot leaves
    // the run as it was
    const uint64_t nv = p->space->n_valid;
    const size_t P = d.P, PD = (size_t)d.P * d.D;
    // the non-aware variant's positions may name no configuration (an invalid one, +inf)
    auto bad_pos = [&](uint32_t v) { return v >= nv && !(d.unaware && v == 0xFFFFFFFFu); };
    if (bad_pos(h[6])) return ct_fail(CT_EINVAL, "ct_pop_restore: best position out of range");
    std::vector<uint32_t> words;
    std::vector<uint8_t> rows;
    std::vector<uint64_t> lin;
    uint32_t pop_best = 0;
    if (d.algo == CT_PSO) {
        const int64_t xmax = (int64_t)d.M * 65536;
        std::vector<int32_t> X(PD), PB(PD);
        std::vector<int64_t> V(PD);
        std::vector<uint32_t> pb_pos(P);
        uint32_t gi;
        memcpy(X.data(), o, PD * 4);
        memcpy(V.data(), o + PD * 4, PD * 8);
        memcpy(PB.data(), o + PD * 12, PD * 4);
        memcpy(pb_pos.data(), o + PD * 16 + P * 4, P * 4);
        memcpy(&gi, o + PD * 16 + P * 8, 4);
        for (size_t k = 0; k < PD; ++k) {
            if (X[k] < 0 || X[k] >= xmax || PB[k] < 0 || PB[k] >= xmax)
                return ct_fail(CT_EINVAL, "ct_pop_restore: particle coordinate outside [0, M * 2^16)");
            // the inertia product w * V (w < 2^16) must stay inside int64
            if (V[k] <= -(1ll << 46) || V[k] >= (1ll << 46))
                return ct_fail(CT_EINVAL, "ct_pop_restore: velocity magnitude not below 2^46");
        }
        for (uint32_t v : pb_pos)
            if (bad_pos(v)) return ct_fail(CT_EINVAL, "ct_pop_restore: personal-best position out of range");
        if (gi >= d.P) return ct_fail(CT_EINVAL, "ct_pop_restore: global-best index out of range");
    } else {
        std::vector<uint32_t> pos(P);
        std::vector<float> f(P);
        memcpy(pos.data(), o, P * 4);
        memcpy(f.data(), o + P * 4, P * 4);
        for (uint32_t v : pos)
            if (bad_pos(v)) return ct_fail(CT_EINVAL, "ct_pop_restore: position out of range");
        if (has_rows(d)) {
            // rows to the device layout (R bytes each) and their linear indices
            const uint8_t* src = o + P * 8;
            const DevSpace& S = p->space->dev;
            rows.assign(P * d.R, 0);
            lin.assign(P, 0);
            for (size_t i = 0; i < P; ++i)
                for (uint32_t j = 0; j < d.D; ++j) {
                    const uint8_t v = src[i * d.D + j];
                    if (v >= S.radix[j]) return ct_fail(CT_EINVAL, "ct_pop_restore: member digit outside its domain");
                    rows[i * d.R + j] = v;
                    lin[i] += (uint64_t)v * S.stride[j];
                }
            // DE's "best" member: lowest objective, then index
            for (uint32_t i = 1; i < d.P; ++i)
                if (f[i] < f[pop_best]) pop_best = i;
        }
        if (d.algo == CT_FIREFLY) {
            const int64_t xmax = (int64_t)d.M * 65536;
            std::vector<int32_t> X(PD);
            memcpy(X.data(), o + P * 8, PD * 4);
            for (int32_t x : X)
                if (x < 0 || x >= xmax) return ct_fail(CT_EINVAL, "ct_pop_restore: firefly coordinate outside [0, M * 2^16)");
        }
        if (d.algo == CT_DE && !d.unaware) {
            // the membership bitmap is derived from the positions, which must be distinct
            words.assign((nv + 31) / 32, 0);
            for (uint32_t v : pos) {
                if (words[v >> 5] & (1u << (v & 31u)))
                    return ct_fail(CT_EINVAL, "ct_pop_restore: DE population holds a configuration twice");
                words[v >> 5] |= 1u << (v & 31u);
            }
        }
    }
    CT_HIP(hipDeviceSynchronize());
    uint32_t stt[4] = {h[4], h[5], d.unaware && d.algo == CT_DE ? pop_best : 0u, 0};
    uint64_t b = ((uint64_t)h[7] << 32) | h[6];
    if (d.algo == CT_PSO) {
        CT_HIP(hipMemcpy(d.X, o, PD * 4, hipMemcpyHostToDevice)); o += PD * 4;
        CT_HIP(hipMemcpy(d.V, o, PD * 8, hipMemcpyHostToDevice)); o += PD * 8;
        CT_HIP(hipMemcpy(d.PB, o, PD * 4, hipMemcpyHostToDevice)); o += PD * 4;
        CT_HIP(hipMemcpy(d.f_pb, o, P * 4, hipMemcpyHostToDevice)); o += P * 4;
        CT_HIP(hipMemcpy(d.pb_pos, o, P * 4, hipMemcpyHostToDevice)); o += P * 4;
        memcpy(&stt[2], o, 4);
    } else {
        CT_HIP(hipMemcpy(d.pos, o, P * 4, hipMemcpyHostToDevice)); o += P * 4;
        CT_HIP(hipMemcpy(d.f, o, P * 4, hipMemcpyHostToDevice)); o += P * 4;
        if (d.algo == CT_FIREFLY) CT_HIP(hipMemcpy(d.X, o, PD * 4, hipMemcpyHostToDevice));
        if (has_rows(d)) {
            CT_HIP(hipMemcpy(d.prow, rows.data(), rows.size(), hipMemcpyHostToDevice));
            CT_HIP(hipMemcpy(d.pL, lin.data(), P * 8, hipMemcpyHostToDevice));
        } else if (d.algo == CT_DE) {
            CT_HIP(hipMemcpy(d.member, words.data(), words.size() * 4, hipMemcpyHostToDevice));
        }
    }
    CT_HIP(hipMemcpy(d.state, stt, 16, hipMemcpyHostToDevice));
    CT_HIP(hipMemcpy(d.best, &b, 8, hipMemcpyHostToDevice));
    if (d.algo == CT_GA) {
        // the rank order the next proposals read is derived from the population
        if (int rc = pop_sort_device(p, nullptr)) return rc;
        CT_HIP(hipDeviceSynchronize());
    }
    return CT_OK;
}

int ct_space_footprint(const ct_space* s, uint64_t* bytes) {
    if (!s || !bytes) return ct_fail(CT_EINVAL, "ct_space_footprint: null argument");
    *bytes = s->dev_bytes;
    return CT_OK;
}

int ct_pop_footprint(const ct_pop* p, uint64_t* bytes) {
    if (!p || !bytes) return ct_fail(CT_EINVAL, "ct_pop_footprint: null argument");
    *bytes = p->dev_bytes + (p->single ? batch_bytes(p->single->cap) : 0);
    return CT_OK;
}

void ct_pop_free(ct_pop* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    batch_free(p->single);
    for (void* q : p->allocs) (void)hipFree(q);
    delete p;
}

}  // extern "C"
