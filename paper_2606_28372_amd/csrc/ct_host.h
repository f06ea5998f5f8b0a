// Host-side internals of libct: handle layouts, device descriptors shared by
// host and kernels, error reporting and the launch entry points of each file.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ct.h"
#include "ct_device.h"

int ct_fail(int code, const std::string& msg);
void prof_suspend(bool on);          // no event records (while a stream is being captured)
// device counters of the boxes and chunks the repair scans open, or null when not counting
unsigned long long* prof_box_counter();

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
    DevSpace dev{};                   // host copy of the device view
    DevSpace* d_dev = nullptr;        // the same view in device memory
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
    uint32_t* d_tab_meta = nullptr;   // scope tables: per program CT_TAB_META words
    uint64_t* d_tabs = nullptr;
    std::vector<uint32_t> tab_meta;       // [2 n_cons][CT_TAB_META]: tables tested, own tables
    uint64_t own_words = 0;               // table words of the programs' own tables (the shared ones follow)
    uint64_t tab_words = 0;
    uint64_t n_ctx = 0;               // combinations of the context parameters (0: no inner patterns)
    size_t lds_values_bytes = 0;      // dynamic LDS for the value tables
    std::vector<uint32_t> code;       // constraint programs, prefix-only ones first
    uint64_t byte_limit = 0;          // build: fail with CT_ENOMEM (n_valid set) if the space would exceed it
    bool over_limit = false;          // the last build stopped at byte_limit
    uint64_t dev_bytes = 0;           // device bytes held once built
};

// Largest table of inner patterns (bits over every context and inner configuration) the build uses.
constexpr uint64_t kPatternBits = 1ull << 27;

// api.cpp: host-side validation and layout, then device build (optionally under a byte limit)
int space_prepare(const int64_t* values, const uint32_t* radices, uint32_t n_params, const uint32_t* code,
                  const uint32_t* cons_offsets, uint32_t n_cons, ct_space** out);
int space_realize(ct_space* s, hipStream_t st, uint64_t byte_limit);

// space.hip
int space_build_device(ct_space* s, hipStream_t st);
uint64_t space_resident_bytes(const ct_space* s, uint64_t n_valid);   // device bytes of the built space
uint64_t space_build_scratch_bytes(const ct_space* s);                // temporaries during the build
int launch_valid_mask(const ct_space* s, const uint8_t* rows, uint64_t n, uint8_t* out, hipStream_t st);
int launch_rank(const ct_space* s, const uint8_t* rows, uint64_t n, int64_t* pos, hipStream_t st);

// ---------------------------------------------------------------------------
// Repair: one RepairSet per (candidate batch, pass); sets live in device
// memory so one launch can serve many runs of different spaces.
// ---------------------------------------------------------------------------
struct RepairSet {
    const DevSpace* S;                // device view of the space
    const uint8_t* rows;              // candidates [n][R]
    uint32_t n;
    uint32_t metric;
    uint64_t seed;
    const uint32_t* gen;              // device generation counter (nullable -> gen_value)
    uint32_t gen_value;
    uint32_t pad0;
    const uint32_t* who;              // nullable: candidate index
    const int32_t* pos_q16;           // TIER_EUCLID positions [n][D]
    uint8_t* out_rows;                // [n][R]
    uint32_t* out_pos;                // [n]
    const uint8_t* apply;             // nullable: per-candidate flag, 0 = leave alone
    uint32_t* list;                   // candidates that need a scan [n]
    uint64_t* list_ins;               // their insertion positions in the valid list (~0: outside the domain) [n]
    uint32_t* fb_list;                // candidates without any tier 0-2 neighbour [n]
    uint64_t* fb_ins;
    uint32_t* count;                  // [0] list length, [1] fallback length
    uint64_t* part_key;               // per (candidate, part) winners [slots]
    uint32_t* part_pos;
    unsigned long long* tally;        // nullable: += candidates scanned
    uint32_t R;                       // copies of the space's row bytes and 64-row box count, so the
    uint32_t pad1;                    // plan reads one descriptor instead of following S
    uint64_t n_sub;
};

// Scan kernels are specialised by (metric, row width): class = metric * 4 + log2(R / 4).
constexpr uint32_t kRepairClasses = 20;
__host__ __device__ inline uint32_t repair_class(uint32_t metric, uint32_t R) {
    return metric * 4u + (R <= 4 ? 0u : R <= 8 ? 1u : R <= 16 ? 2u : 3u);
}

// Device-side plan of one scan pass over a set array (written by the last block of the kernel
// before the scans: proposal, preparation or main finish).
struct RepairPlan {
    uint32_t* cand_off;               // [n_sets + 1] prefix of candidate counts
    uint32_t* item_off;               // [kRepairClasses][n_sets + 1] prefix of (candidate, part) items per class
    uint32_t* parts;                  // [n_sets]
    uint32_t* done;                   // blocks finished in the kernel that plans (0 between launches)
    unsigned long long* opened;       // nullable (measurement): [which * 2] += 64-row boxes opened,
                                      // [which * 2 + 1] += chunks opened, over the pass's scan items
};

constexpr uint32_t kRepairTargetWaves = 8192;   // scan items per class launch, untuned (ct_repair's slot minimum)
// Largest item target a batch may be tuned to; every run holds max(P, kRepairMaxItems) slots for
// per-(candidate, part) winners, so c candidates of a set split into p parts (c * p <= the target,
// or p = 1) always fit.
constexpr uint32_t kRepairMaxItems = 32768;

// How the scan classes of one pass are launched: one after another, side by side on the fan's
// streams, or the scanned metrics of one row width together in one launch.
constexpr uint32_t kScanSerial = CT_SCAN_SERIAL, kScanStreams = CT_SCAN_STREAMS, kScanFused = CT_SCAN_FUSED;

// Work partitioning of the scan launches (chosen by the autotuner; results do not depend on it):
// items per class (candidates x parts), least 64-row boxes per part, waves in the grid, and how
// the classes are launched.
struct RepairTune {
    uint32_t items = kRepairTargetWaves;
    uint32_t min_sub = 32;
    uint32_t grid_waves = 8192;
    uint32_t mode = kScanSerial;
};

// Auxiliary streams (default priority) on which the independent scan classes of one pass run
// side by side: fork after the plan, join before the finish.  Three lanes plus the launch stream
// fit the four hardware queues a process gets by default.
struct StreamFan {
    static constexpr int kLanes = 3;
    hipStream_t s[kLanes] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kLanes] = {};
};
int fan_create(StreamFan* f);
void fan_destroy(StreamFan* f);

// Host helpers to run a repair pass sequence over a device set array.
struct RepairPasses {
    RepairTune tune;
    StreamFan* fan = nullptr;               // nullable: run the scan classes one after another
    uint32_t n_sets = 0;
    const RepairSet* d_sets = nullptr;
    const uint32_t* d_prep_off = nullptr;   // [n_sets + 1] prefix of n
    uint32_t total_n = 0;
    uint32_t class_mask = 0;                // scan classes of the main pass (bit per repair_class)
    uint32_t fb_class_mask = 0;             // Hamming classes of the fallback pass of tiered sets (0: none)
    uint32_t euclid_tab = 0;                // largest max_radix * (R + 1) over TIER_EUCLID sets (LDS table entries)
    RepairPlan plan{};
};
int repair_plan_alloc(RepairPlan& p, uint32_t n_sets, std::vector<void*>& owned);
struct PlanArgs;
PlanArgs main_plan(const RepairPasses& rp);   // what plans the main scans of a pass
// prep + scan + finish (+ Hamming fallback for tiered metrics); `zero_counts` clears the
// sets' counters with a kernel first (the step sequence clears them in its selection kernel);
// prep = false when the candidates were already listed and the main scans planned (the step's
// propose kernel does both).
int launch_repair_passes(const RepairPasses& rp, bool zero_counts, hipStream_t st, bool count_tally = true,
                         bool prep = true);
// GA mutation of the flagged children of a HAM1_RANDOM set array, in place, one kernel
int launch_mutation(const RepairPasses& rp, hipStream_t st);
// clear the sets' counters and list their candidates (validity, rank, list), without a plan
int launch_repair_prep(const RepairPasses& rp, hipStream_t st);
// Repair by enumeration of neighbour shells through the bitmask, then the scans for what it left:
// `listed` is prepared (its candidates listed), enumeration settles what it can within
// max_lookups bitmask lookups per candidate and lists the rest in `rest` (the same sets with
// their own list and counters), whose scans then run.  d_stats (nullable): settled, lookups.
int launch_repair_enum(const RepairPasses& listed, const RepairPasses& rest, uint64_t max_lookups,
                       unsigned long long* d_stats, hipStream_t st);

// ---------------------------------------------------------------------------
// Optimiser runs
// ---------------------------------------------------------------------------
struct PopDev {
    const DevSpace* S;                // device view of the run's space
    uint32_t algo, P, D, R;
    uint64_t seed;
    uint32_t F_q16, de_method;
    uint32_t de_cross, ga_cross;      // DE: binomial / exponential; GA: crossover operator
    uint32_t unaware;                 // the non-constraint-aware variant
    uint8_t* prow;                    // non-aware DE/GA: member rows [P][R] (members may be invalid)
    uint64_t* pL;                     // non-aware DE/GA: member linear indices [P]
    uint64_t* tL;                     // non-aware DE: trial linear indices [P] (selection scratch)
    uint64_t CR_q32;
    int64_t w_q16, c1_q16, c2_q16;
    uint64_t mut_thresh;              // floor(2^32 / mutation_chance): a child mutates when its draw is below
    uint32_t M;                       // largest radix (PSO/Firefly domain [0, M) per dimension)
    int64_t ff_B0, ff_gamma, ff_alpha;  // Firefly B0, gamma, alpha in Q16.16
    uint64_t n_valid;
    const float* obj;                 // [n_valid]
    uint32_t* state;                  // [0] generation, [1] reinits, [2] gbest index, [3] accepted
    uint64_t* best;                   // packed (orderable float bits << 32) | position
    uint32_t* pos;                    // [P] population (DE/GA) as valid-list positions; Firefly: evaluated position
    float* f;                         // [P] objective (Firefly: brightness, lower is brighter)
    uint8_t* trial;                   // [P][R] proposals
    uint8_t* out;                     // [P][R] after repair (and mutation)
    uint32_t* tpos;                   // [P] positions of `out`
    uint8_t* apply;                   // [P] GA mutation flags
    uint32_t* member;                 // DE: bitmap over valid positions
    uint32_t* claim;                  // DE: [n_valid] lowest accepted trial index per position
    uint32_t* sorted;                 // GA: positions by rank
    const uint64_t* beta;             // GA: cumulative selection thresholds [P]
    int32_t* X;                       // PSO / Firefly [P][D] Q16.16 positions
    int32_t* Xn;                      // Firefly [P][D] positions after this generation's moves
    int64_t* V;                       // PSO [P][D] velocities
    int32_t* PB;                      // PSO [P][D] personal-best positions
    float* f_pb;                      // PSO [P]
    uint32_t* pb_pos;                 // PSO [P]
    unsigned long long* tally;        // [0] repair scans, [1] mutation scans (cumulative)
    uint32_t* rcount;                 // [4] repair counters: main pass, fallback, mutation pass, spare
};

struct ct_batch;

struct ct_pop {
    const ct_space* space = nullptr;
    ct_pop_params prm{};
    PopDev dev{};
    std::vector<void*> allocs;
    uint64_t dev_bytes = 0;           // device bytes of the run's own buffers
    ct_batch* single = nullptr;       // batch of this run alone (plain stepping)
    // repair scratch of this run
    uint32_t* r_list = nullptr;
    uint64_t* r_list_ins = nullptr;
    uint32_t* r_fb = nullptr;
    uint64_t* r_fb_ins = nullptr;
    uint64_t* r_part_key = nullptr;
    uint32_t* r_part_pos = nullptr;
};

// A group of runs stepped together: descriptor arrays in device memory (sized for `cap`
// runs, refilled in place when the group changes) and, once captured, a graph.
struct ct_batch {
    std::vector<ct_pop*> pops;
    uint32_t n = 0, cap = 0;
    PopDev* d_pops = nullptr;
    uint32_t* d_ind_off = nullptr;    // [n + 1] prefix of population sizes
    uint32_t* d_ga_off = nullptr;     // [n_ga + 1] prefix of GA population sizes
    uint32_t* d_ff_off = nullptr;     // [n + 1] prefix of Firefly population sizes (0 for other runs)
    RepairSet* d_setsA = nullptr;
    RepairSet* d_setsC = nullptr;
    uint32_t total_ind = 0;
    uint32_t n_ga = 0, max_pop = 0;
    uint32_t total_ff = 0;            // fireflies in the group
    RepairPasses passA, passC;        // main repair, GA mutation
    std::vector<void*> owned;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string shape;                // signature of the group for the tuning cache
    bool tuned = false;
    std::vector<RepairTune> tune_cand;   // autotuner: candidate partitionings
    std::vector<double> tune_ms;         // their pass times summed over the tuning generations
    StreamFan fan;
    // Lanes: the runs split into sub-batches (run i in lane i mod lanes), each stepped on a stream
    // of its own, so that one lane's phases run while another's wait at a phase boundary (by
    // default kLanes of them for groups of kLaneMinRuns runs or more).  The group's own descriptor
    // arrays are then left empty.
    std::vector<ct_batch*> lanes;
    std::vector<hipStream_t> lane_st;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t lane_fork = nullptr;
};

constexpr uint32_t kLaneMinRuns = 64;
constexpr uint32_t kLanes = 2;
constexpr uint32_t kMaxLanes = 8;

// Smallest DE population for a mutation operator (i and its distinct picks).
inline uint32_t de_min_pop(uint32_t method) { return method == CT_DE_RAND2 || method == CT_DE_BEST2 ? 6u : 4u; }

// Device bytes a run of this shape allocates (its buffers and its one-run batch).
uint64_t pop_footprint_bytes(uint32_t algo, uint32_t P, uint32_t D, uint32_t R, uint64_t n_valid, uint32_t unaware);

// step.hip
int pop_init_device(ct_pop* p, hipStream_t st);
// GA: the population's rank order (after creation or a restore; generations keep it current)
int pop_sort_device(ct_pop* p, hipStream_t st);
int batch_generation(ct_batch* b, hipStream_t st);
// n_generations generations; every sample_every-th sweeps the main repair pass over the candidate
// partitionings, those in between decide the side-stream setting; installs the choice
int batch_autotune(ct_batch* b, uint32_t n_generations, uint32_t sample_every, hipStream_t st);

// api.cpp
int batch_build(const std::vector<ct_pop*>& pops, ct_batch** out, hipStream_t st);
// refill a batch with another group of runs (reallocating only if it outgrows the capacity);
// the caller makes sure no launch that reads the old descriptors is still pending
int batch_fill(ct_batch* b, const std::vector<ct_pop*>& pops);
void batch_free(ct_batch* b);
