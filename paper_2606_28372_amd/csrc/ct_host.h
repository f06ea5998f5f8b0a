// Host-side internals of libct: handle layouts, error reporting, launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ct.h"
#include "ct_device.h"

int ct_fail(int code, const std::string& msg);

// Records HIP events around the enclosed launch when kernel timing is enabled.
class ProfScope {
  public:
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
  private:
    const char* name_;
    hipStream_t st_;
    void* a_;
};

#define CT_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ct_fail(CT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

struct ct_space {
    DevSpace dev{};                   // device view handed to kernels
    uint32_t D = 0, R = 0, n_cons = 0;
    std::vector<int64_t> values;
    std::vector<uint32_t> radices;
    uint64_t n_cartesian = 0, n_valid = 0, n_words = 0;
    int device = 0;
    int64_t* d_values = nullptr;
    uint32_t* d_code = nullptr;
    uint64_t* d_prefix = nullptr;
    uint64_t* d_words = nullptr;
    uint64_t* d_lin = nullptr;
    uint8_t* d_rows = nullptr;
    uint8_t* d_prevnext = nullptr;
    uint64_t* d_grp_off = nullptr;
    uint16_t* d_dir8 = nullptr;
    uint8_t* d_boxes = nullptr;
    size_t lds_values_bytes = 0;      // dynamic LDS for the value tables
};

// space.hip
int space_build_device(ct_space* s, hipStream_t st);
int launch_valid_mask(const ct_space* s, const uint8_t* rows, uint64_t n, uint8_t* out, hipStream_t st);
int launch_rank(const ct_space* s, const uint8_t* rows, uint64_t n, int64_t* pos, hipStream_t st);

// Per-candidate repair job description shared by ct_repair and the optimiser steps.
struct RepairJob {
    const DevSpace* S_host;           // host copy of the space view (for launch shapes)
    DevSpace S;                       // passed to kernels
    const uint8_t* rows;              // candidates [n][R]
    uint64_t n;
    uint32_t metric;
    uint64_t seed;
    const uint32_t* d_gen;            // device generation counter (nullable -> gen_value)
    uint32_t gen_value;
    const uint32_t* who;              // nullable: candidate index
    const int32_t* pos_q16;           // TIER_EUCLID positions [n][D]
    uint8_t* out_rows;
    uint32_t* out_pos;
    const uint8_t* apply;             // nullable: per-candidate flag, 0 = leave alone (still written)
    unsigned long long* tally;        // nullable: += number of candidates scanned
};

struct RepairScratch {
    uint32_t* list = nullptr;         // candidates that need a scan, then the fallback list [2][cap]
    uint64_t* list_L = nullptr;       // their linear indices [2][cap]
    uint32_t* count = nullptr;        // [2]: list length, fallback length
    uint64_t* part_key = nullptr;     // per (candidate, part) best key
    uint32_t* part_pos = nullptr;     // per (candidate, part) best position
    uint64_t cap = 0;
    uint32_t max_parts = 0;
};

int repair_scratch_alloc(RepairScratch& rs, uint64_t cap, uint32_t max_parts, hipStream_t st);
void repair_scratch_free(RepairScratch& rs, hipStream_t st);
int launch_repair(const ct_space* s, const RepairJob& job, RepairScratch& rs, hipStream_t st);

// One optimiser run's device view (kernel argument).
struct PopDev {
    DevSpace S;
    uint32_t algo, P, D, R;
    uint64_t seed;
    uint32_t F_q16, de_best;
    uint64_t CR_q32;
    int64_t w_q16, c1_q16, c2_q16;
    uint32_t mut_thresh;              // floor(2^32 / mutation_chance)
    uint32_t M;                       // largest radix (PSO domain [0, M) per dimension)
    const float* obj;                 // [n_valid]
    uint32_t* state;                  // [0] generation, [1] reinits, [2] gbest index, [3] accepted
    uint64_t* best;                   // packed (float bits << 32) | position
    uint32_t* pos;                    // [P] population (DE/GA) as valid-list positions
    float* f;                         // [P]
    uint8_t* trial;                   // [P][R] proposals
    uint8_t* out;                     // [P][R] after repair (and mutation)
    uint32_t* tpos;                   // [P] positions of `out`
    uint8_t* apply;                   // [P] GA mutation flags
    uint32_t* member;                 // DE: bitmap over valid positions
    uint32_t* claim;                  // DE: [n_valid] lowest accepted trial index per position
    uint32_t* sorted;                 // GA: positions by rank
    const uint64_t* beta;             // GA: cumulative selection thresholds [P]
    int32_t* X;                       // PSO [P][D] Q16.16 positions
    int64_t* V;                       // PSO [P][D] velocities
    int32_t* PB;                      // PSO [P][D] personal-best positions
    float* f_pb;                      // PSO [P]
    uint32_t* pb_pos;                 // PSO [P]
    unsigned long long* tally;        // [0] repair scans, [1] mutation scans (cumulative)
};

struct ct_pop {
    const ct_space* space = nullptr;
    ct_pop_params prm{};
    PopDev dev{};
    RepairScratch rs;
    std::vector<void*> allocs;
};

// step.hip
int pop_init_device(ct_pop* p, hipStream_t st);
int pop_step_plain(ct_pop* p, hipStream_t st);
