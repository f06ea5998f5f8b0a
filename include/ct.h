/*
 * ct.h -- C ABI of the MI355X constraint-aware auto-tuning library (libct.so).
 *
 * The library implements, on one gfx950 GPU, the data-parallel hot path of
 * constraint-aware evolutionary auto-tuning (Willemsen et al.,
 * "Constraint-aware Optimization in Auto-Tuning"):
 *   - evaluating the correctness constraints of a discrete tunable-parameter
 *     space (the CSP (X, D, C) of Section IV-A) over every configuration,
 *     giving a validity bitmask and the ascending list of valid
 *     configurations (Section IV-A: the full space is resolved before tuning);
 *   - validity queries and repair of invalid configurations to a valid one
 *     under the neighbour rules of Section IV-A (Alg. 1 Repair, Alg. 2, Alg. 3);
 *   - whole-population generation steps of constraint-aware Differential
 *     Evolution (Alg. 1, Section IV-B), Particle Swarm Optimization
 *     (Section IV-C) and the Genetic Algorithm (Section IV-D).
 *
 * Conventions
 *   - Every function returns CT_OK (0) or a negative ct_status; on error
 *     nothing is written to caller buffers and ct_last_error() returns a
 *     message for the calling thread.
 *   - "d_" pointers are device pointers on the current HIP device (for
 *     example torch tensors' data_ptr()); "h_" pointers are host memory.
 *     The caller owns every buffer it passes; handles own their internal
 *     device buffers and release them in the matching *_free.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered and asynchronous unless stated otherwise.
 *   - A configuration is a row of value indices ("digits"), one uint8 per
 *     parameter, padded with zeros to row_bytes = 4, 8, 16 or 32 bytes
 *     (D <= 4, 8, 16, 32).  Its linear index is row-major with the last
 *     parameter fastest: L = sum_j d_j * prod_{k>j} r_k.
 *   - Randomness is Philox4x32-10 (Salmon et al., SC'11) keyed by a 64-bit
 *     seed at counters that name each draw, so results are bit-exact and
 *     independent of launch shape, batching and stream interleaving.
 */
#ifndef CT_H
#define CT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ct_space ct_space;   /* a resolved search space (device-resident) */
typedef struct ct_pop ct_pop;       /* one optimiser run's device state */

enum ct_status {
    CT_OK = 0,
    CT_EINVAL = -1,     /* bad argument, malformed bytecode, unsupported size */
    CT_ENOMEM = -2,     /* device allocation failed */
    CT_EOVERFLOW = -3,  /* a constraint may overflow 64-bit integers */
    CT_EEMPTY = -4,     /* repair/step on a space with no valid configuration */
    CT_EDEVICE = -5,    /* HIP runtime error */
    CT_ESYNTAX = -6     /* constraint text not in the accepted expression language */
};

/* Repair keys (Section IV-A neighbour rules).  Ties always go to the lowest linear index. */
enum ct_metric {
    CT_HAMMING = 0,      /* number of differing parameters ("Hamming") */
    CT_INDEX_L1 = 1,     /* sum of |index differences| ("index-distance"; DE repair, Alg. 1) */
    CT_TIER_EUCLID = 2,  /* first non-empty of strictly-adjacent / adjacent / Hamming-1, nearest to a
                            continuous position by Euclidean distance (PSO, Alg. 2) */
    CT_TIER_RANDOM = 3,  /* same sets, uniformly random member (GA, Alg. 3) */
    CT_HAM1_RANDOM = 4   /* uniformly random valid Hamming-1 neighbour (GA mutation, Section IV-D) */
};

enum ct_algo { CT_DE = 0, CT_PSO = 1, CT_GA = 2, CT_FIREFLY = 3 };

enum ct_step_flags {
    CT_STEP_PLAIN = 0,    /* each population advanced by its own launch sequence */
    CT_STEP_BATCHED = 1,  /* all populations advanced together, one launch per phase */
    CT_STEP_GRAPH = 2     /* BATCHED, captured once into a hipGraph and replayed per generation */
};

#define CT_MAX_PARAMS 32
#define CT_MAX_RADIX 255
#define CT_MAX_POP 65536
#define CT_UNAWARE_DE_MAX_POP 8192   /* non-aware DE: its selection compares every pair of members */
#define CT_MAX_CARTESIAN_LOG2 46
/* Valid-list positions are 32-bit (0xFFFFFFFF means "none"): ct_repair, ct_pop_create and the
   server need n_valid <= CT_MAX_VALID; larger spaces still build, count, mask and rank. */
#define CT_MAX_VALID 0xFFFFFFFEull

/* Message for the last error on this thread (never NULL). */
const char* ct_last_error(void);

/* Library ABI version (currently 2: ct_pop_params carries the Firefly parameters and the
   DE / GA operator choices). */
int ct_version(void);

/*
 * ct_compile -- constraint text -> integer expression bytecode (host only, no GPU).
 *
 * Section IV-A defines each constraint as a predicate over a subset of the
 * parameters; here a constraint is a Python integer expression over the
 * parameter names: integer literals, True/False, + - * // %, unary - and +,
 * abs(x), min(a, b, ...), max(a, b, ...), comparisons (chains allowed),
 * and / or / not, parentheses.  Semantics are Python's: floor division,
 * modulo with the sign of the divisor, 'and'/'or' return an operand, a
 * division or modulo by zero makes the whole constraint false (where Python
 * would raise), and a configuration is valid iff every constraint is truthy.
 * Interval analysis over the value tables must prove every intermediate fits
 * in int64 (else CT_EOVERFLOW).
 *
 *   names[n_params], values (concatenated value lists), radices[n_params]
 *   constraints[n_cons]: NUL-terminated strings
 *   code[code_cap]: output words; cons_offsets[n_cons + 1]: start of each program
 *   *code_len: words written.
 * Errors: CT_ESYNTAX (message names the constraint and position),
 *         CT_EOVERFLOW, CT_EINVAL (sizes, unknown name, capacity too small).
 */
int ct_compile(const char* const* names, uint32_t n_params, const int64_t* values, const uint32_t* radices,
               const char* const* constraints, uint32_t n_cons,
               uint32_t* code, uint32_t code_cap, uint32_t* cons_offsets, uint32_t* code_len);

/*
 * ct_space_build -- resolve the whole space on the GPU (Section IV-A).
 *
 * Decodes every linear index L in [0, prod r_j), evaluates every constraint
 * program, writes the validity bitmask (bit L%64 of word L/64) and compacts
 * the valid configurations into an ascending list of linear indices plus
 * their digit rows.  Inputs are host arrays copied into the handle.
 *   1 <= n_params <= 32, 1 <= r_j <= 255, prod r_j < 2^46.
 * Errors: CT_EINVAL (sizes, malformed bytecode: unknown opcode, stack
 * under/overflow, parameter id out of range), CT_ENOMEM, CT_EDEVICE.
 * An empty valid set is not an error (count 0).
 */
int ct_space_build(const int64_t* values, const uint32_t* radices, uint32_t n_params,
                   const uint32_t* code, const uint32_t* cons_offsets, uint32_t n_cons,
                   void* stream, ct_space** out);

/* Number of valid and of all configurations.  Synchronises with the build. */
int ct_space_count(const ct_space* s, uint64_t* n_valid, uint64_t* n_cartesian);

/* Number of parameters and the row width in bytes. */
int ct_space_info(const ct_space* s, uint32_t* n_params, uint32_t* row_bytes);

/* Borrowed device pointers (valid until ct_space_free): ascending linear indices
   [n_valid] and digit rows [n_valid][row_bytes]. */
int ct_space_valid_list(const ct_space* s, const uint64_t** d_lin, const uint8_t** d_rows);

/* Borrowed device pointer to the validity bitmask [ceil(n_cartesian/64)] words. */
int ct_space_bitmask(const ct_space* s, const uint64_t** d_words, uint64_t* n_words);

/* Stream-ordered device-to-device copies of the valid list / bitmask into
   caller-owned buffers: d_lin[n_valid] (nullable), d_rows[n_valid][row_bytes]
   (nullable); d_words[ceil(n_cartesian/64)]. */
int ct_space_copy_list(const ct_space* s, uint64_t* d_lin, uint8_t* d_rows, void* stream);
int ct_space_copy_bitmask(const ct_space* s, uint64_t* d_words, void* stream);

void ct_space_free(ct_space* s);

/*
 * ct_valid_mask -- is each row a solution (Section IV-A validity query)?
 *   d_rows[n][row_bytes] -> d_out[n] (1 valid, 0 invalid; a digit >= its
 *   radix counts as invalid).
 */
int ct_valid_mask(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint8_t* d_out, void* stream);

/*
 * ct_rank -- position of each row in the ascending valid list, or -1 if the
 * row is not valid.  d_rows[n][row_bytes] -> d_pos[n] (int64).
 */
int ct_rank(const ct_space* s, const uint8_t* d_rows, uint64_t n, int64_t* d_pos, void* stream);

/*
 * ct_repair -- move invalid rows to a valid configuration.
 *
 * For metrics HAMMING, INDEX_L1, TIER_EUCLID and TIER_RANDOM a valid row is
 * returned unchanged; an invalid row c becomes the valid v minimising the
 * lexicographic key (k(c, v), L(v)):
 *   HAMMING      k = #differing parameters
 *   INDEX_L1     k = sum_j |v_j - c_j|
 *   TIER_*       k = (tier, sub): tier 0 strictly adjacent (every |v_j - c_j| <= 1),
 *                1 adjacent (every v_j is c_j or the nearest lower/higher value index of
 *                parameter j that occurs in some solution), 2 Hamming-1, 3 otherwise;
 *                sub = squared distance between the particle position X (Q16.16 index
 *                units, d_pos_q16[n][n_params]) and the value centres (2 v_j + 1) * 2^15
 *                for TIER_EUCLID, or a Philox draw at counter
 *                (who, generation, 7<<24 | L>>32, L & 0xffffffff) for TIER_RANDOM;
 *                in tier 3 sub is the Hamming distance.
 * HAM1_RANDOM applies to every row: it becomes the valid Hamming-1 neighbour
 * with the smallest Philox draw at counter (who, generation, 8<<24 | L>>32, L),
 * or stays unchanged if it has none.
 *   d_who[n] (nullable: row index) is the counter word naming each row.
 * Outputs: d_out_rows[n][row_bytes], d_out_pos[n] (position of the result in
 * the valid list, or 0xFFFFFFFF for an unchanged invalid HAM1_RANDOM row).
 * d_out_rows may equal d_rows.
 * Errors: CT_EEMPTY (no valid configuration), CT_EINVAL (also n_valid > CT_MAX_VALID), CT_ENOMEM.
 */
int ct_repair(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric,
              uint64_t seed, uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16,
              uint8_t* d_out_rows, uint32_t* d_out_pos, void* stream);

/*
 * ct_repair_enum -- ct_repair by enumeration of neighbour shells through the validity bitmask
 * (Section IV-A: with the space resolved, whether a configuration is valid is one bit), with
 * the scans for what enumeration leaves; the results are ct_repair's, bit for bit.
 *
 * For an invalid in-domain row c the shells are visited in the order of the metric's leading
 * key, and the first shell holding a valid configuration holds the winner:
 *   HAMMING      Hamming spheres of radius 1, 2, ..., 8 around c;
 *   INDEX_L1     index-distance spheres of radius 1, 2, ..., 8;
 *   TIER_*       the strictly-adjacent box (every v_j in {c_j - 1, c_j, c_j + 1}), the adjacent
 *                box (every v_j in {c_j, nearest present value below / above}), the Hamming-1
 *                sphere, then Hamming spheres of radius 2, ..., 8 (Alg. 2 / Alg. 3's sets in order).
 * A shell costs one bitmask lookup per member and is counted before it is visited: rows whose
 * next shell would take their lookups past max_lookups (0: none enumerated), rows outside the
 * domain, rows needing a sphere beyond radius 8, and every HAM1_RANDOM row go through the scans.
 *   h_stats (nullable, host): [0] rows settled by enumeration, [1] lookups spent.  Synchronises.
 * Other arguments, outputs and errors as ct_repair.
 */
int ct_repair_enum(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric,
                   uint64_t seed, uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16,
                   uint64_t max_lookups, uint8_t* d_out_rows, uint32_t* d_out_pos, uint64_t* h_stats,
                   void* stream);

/*
 * ct_repair_noalloc -- ct_repair for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid the
 * allocator).  Same arguments, kernels and results as ct_repair; it calls no
 * device or host allocator.  Its scratch (candidate lists, per-part winners,
 * the set descriptor and the scan plan) is one static device array of
 * CT_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU until
 * the process ends, so n <= CT_NOALLOC_MAX_ROWS (else CT_EINVAL, nothing
 * launched).  The call is stream-ordered and does not synchronise.  Every call
 * on one GPU shares that array (each call clears what it needs first): calls
 * that overlap on one GPU -- on different streams or threads without ordering
 * between them -- race and give undefined results.  The space must live on
 * the current device.
 */
#define CT_NOALLOC_MAX_ROWS 16384u
#define CT_NOALLOC_SCRATCH_BYTES (640u * 1024u)
int ct_repair_noalloc(const ct_space* s, const uint8_t* d_rows, uint64_t n, uint32_t metric,
                      uint64_t seed, uint32_t generation, const uint32_t* d_who, const int32_t* d_pos_q16,
                      uint8_t* d_out_rows, uint32_t* d_out_pos, void* stream);

/*
 * Optimiser hyperparameters in integer form (Table IV defaults in brackets).
 *   DE:  F_q16 = round(F * 2^16) [45875], CR_q32 = round(CR * 2^32) [2576980378],
 *        de_method: mutation operator (Alg. 1 and Section IV-B, last paragraph) [CT_DE_BEST1],
 *        de_crossover: CT_DE_BIN (binomial, Alg. 1) or CT_DE_EXP (exponential) [CT_DE_BIN];
 *        requires pop_size >= 4 (>= 6 for the two-difference operators).
 *   PSO: w_q16 < 65536, c1_q16, c2_q16 <= 2^20  [32768, 196608, 32768].
 *   GA:  mutation_chance X = "one in X" [5]; rank selection Beta(1, beta_b), 1 <= beta_b <= 5 [3];
 *        ga_crossover: CT_GA_SINGLE_POINT [default], CT_GA_TWO_POINT, CT_GA_UNIFORM,
 *        CT_GA_DISRUPTIVE_UNIFORM (Section IV-D).
 *   Firefly (Section IV-C, last paragraph; Table IV): ff_B0_q16 = round(B0 * 2^16) [65536],
 *        ff_gamma_q16 = round(gamma * 2^16) [65536], ff_alpha_q16 = round(alpha * 2^16) [13107],
 *        each <= 2^20.  Positions use PSO's index-unit mapping and Alg. 2 evaluation.
 * Every constraint-aware algorithm requires pop_size <= n_valid (its initial sample is
 * stratified over the valid list, one stratum per member).  Fields a run does not use are
 * ignored; reserved words must be 0.
 *   unaware = 1 selects the non-constraint-aware variant (Sections IV-B and IV-C, last
 * sentences): the initial population is drawn over the whole Cartesian space (digit j of
 * member i: word j%4 of draw (i, 0, 1<<24 | 1 + j/4, 0), uniform over the parameter's values;
 * PSO / Firefly coordinates uniform in [0, M 2^16) from the same words), nothing is repaired,
 * and an invalid configuration evaluates to +infinity (its position is 0xFFFFFFFF).  DE's
 * "best" is then the population's best member (lowest objective, then index); GA ranks by
 * (objective, index) and mutates one parameter (word 1 of the mutation draw) to another of its
 * values (word 2).  Non-aware DE takes pop_size <= CT_UNAWARE_DE_MAX_POP.
 */
typedef struct {
    uint32_t algo;
    uint32_t pop_size;
    uint64_t seed;
    uint32_t F_q16;
    uint32_t de_method;
    uint64_t CR_q32;
    uint32_t w_q16, c1_q16, c2_q16;
    uint32_t mutation_chance;
    uint32_t beta_b;
    uint32_t ff_B0_q16, ff_gamma_q16, ff_alpha_q16;
    uint32_t de_crossover, ga_crossover;
    uint32_t unaware;       /* 1: the non-constraint-aware variant [0] */
    uint32_t reserved[4];
} ct_pop_params;

/* DE mutation operators on value indices, with picks r1..r5 distinct members other than i
   (Philox words 0-2 of draw (i, g, 2<<24, 0), words 0-1 of (i, g, 2<<24 | 1, 0)) and
   m = clip(round_half_up(base + F * difference)):
     RAND1: x_r1 + F (x_r2 - x_r3)             BEST1: best + F (x_r2 - x_r3)
     RAND2: x_r1 + F (x_r2 - x_r3 + x_r4 - x_r5)   BEST2: best + F (x_r2 - x_r3 + x_r4 - x_r5)
     CURRENTTOBEST1: x_i + F (best - x_i + x_r2 - x_r3)
     RANDTOBEST1: x_r1 + F (best - x_r1 + x_r2 - x_r3)
   Exponential crossover takes the mutant on the circular run of coordinates from j_rand that
   continues while draw k (word k%4 of (i, g, 3<<24 | k/4, 0)), k = 1, 2, ..., is below CR.
   GA crossovers of parents A, B (child 2k; child 2k+1 is the mirror): SINGLE_POINT A[:c]+B[c:];
   TWO_POINT A[:c1]+B[c1:c2]+A[c2:] (cuts from words 2 and 3 of the selection draw, distinct);
   UNIFORM gene j from B when the top bit of word j%4 of (k, g, 10<<24 | j/4, 0) is set;
   DISRUPTIVE_UNIFORM: of the genes where A and B differ, the half (rounded down) with the
   smallest keys (word j%4 of (k, g, 10<<24 | j/4, 1), ties by j) come from B. */
enum { CT_DE_RAND1 = 0, CT_DE_BEST1 = 1, CT_DE_RAND2 = 2, CT_DE_BEST2 = 3, CT_DE_CURRENTTOBEST1 = 4,
       CT_DE_RANDTOBEST1 = 5 };
enum { CT_DE_BIN = 0, CT_DE_EXP = 1 };
enum { CT_GA_SINGLE_POINT = 0, CT_GA_TWO_POINT = 1, CT_GA_UNIFORM = 2, CT_GA_DISRUPTIVE_UNIFORM = 3 };

/*
 * ct_pop_create -- allocate a run and draw its initial population (generation 0).
 * d_objective[n_valid] (float32, > 0, borrowed: must outlive the run) stands
 * for the measured runtime of each valid configuration, indexed by position
 * in the valid list; lower is better.
 * Errors: CT_EINVAL (parameters, n_valid > CT_MAX_VALID), CT_EEMPTY, CT_ENOMEM.
 */
int ct_pop_create(const ct_space* s, const ct_pop_params* p, const float* d_objective, void* stream,
                  ct_pop** out);

/*
 * ct_step -- advance n_pops runs by n_generations generations each.
 * DE (Alg. 1): mutate, binomial crossover, INDEX_L1 repair, greedy selection
 * with "u not in X", reinitialisation after a generation without change.
 * PSO (Section IV-C): velocity/position update in Q16.16 index units,
 * snap, TIER_EUCLID evaluation (position unchanged), personal/global best.
 * GA (Section IV-D): sort, Beta rank selection, single-point crossover,
 * TIER_RANDOM repair, HAM1_RANDOM mutation with chance 1/mutation_chance.
 * Firefly (Section IV-C, last paragraph): each firefly moves towards every
 * firefly that was brighter (lower objective) at the start of the generation,
 * in ascending index, by B0 exp(-gamma r^2) of the way (r in PSO's [0,1]^N
 * coordinates; exp in Q0.32 as a product of rounded e^(-2^(b-16)) factors
 * over the set bits b of gamma r^2 in Q16.16) plus alpha (u - 1/2) M per
 * dimension (u from a Philox draw at (i, generation, 9<<24 | d/4, j)), is
 * clamped to [0, M 2^16), then snapped and evaluated through TIER_EUCLID
 * (position unchanged); brightness is the evaluated objective.
 * Results do not depend on `flags`.  Runs may belong to different spaces.
 */
int ct_step(ct_pop* const* pops, uint32_t n_pops, uint32_t n_generations, uint32_t flags, void* stream);

/*
 * Batches: a fixed group of runs (of any spaces and algorithms) advanced
 * together with one launch per phase of the generation for all of them.
 * ct_batch_step with CT_STEP_GRAPH captures one generation into a hipGraph on
 * first use and replays it n_generations times (the generation counters live
 * on the device, so replays need no host work); CT_STEP_BATCHED launches the
 * same kernels directly.  Results equal those of stepping each run alone.
 * The runs must outlive the batch; a run may be in several batches but only
 * one of them may be stepped at a time.  At most 4096 runs per batch.
 * A batch of 64 runs or more is stepped as two lanes (ct_batch_create_lanes
 * chooses the number): run i goes to lane i mod lanes, and each lane
 * advances on a stream of its own (forked from
 * `stream` at the call and joined back into it before the call's work on
 * `stream` completes), so that one lane's phases run while the other's wait at
 * a phase boundary.  ct_batch_autotune tunes the lanes one after the other,
 * ct_batch_set_tuning installs the partitioning in all, and ct_batch_tuning
 * reports the first lane's.
 */
typedef struct ct_batch ct_batch;
int ct_batch_create(ct_pop* const* pops, uint32_t n_pops, ct_batch** out);
/* The same with an explicit number of lanes (1: none; at most 8, and at most one per run).
   CT_EINVAL for 0 or more than 8. */
int ct_batch_create_lanes(ct_pop* const* pops, uint32_t n_pops, uint32_t n_lanes, ct_batch** out);
int ct_batch_step(ct_batch* b, uint32_t n_generations, uint32_t flags, void* stream);
void ct_batch_free(ct_batch* b);

/* How the repair scan classes of one pass are launched (results never depend on it). */
#define CT_SCAN_SERIAL 0u          /* one launch per (metric, row width), one after another */
#define CT_SCAN_STREAMS 1u         /* those launches side by side on auxiliary streams */
#define CT_SCAN_FUSED 2u           /* the scanned metrics of one row width in a single launch */

/*
 * ct_batch_autotune -- advance the batch by exactly n_generations generations,
 * choosing the work partitioning of its repair scans: items per class launch
 * (candidates x list parts), least 64-row boxes per part, waves in the grid,
 * and the launch mode (CT_SCAN_*).  Generations 0, sample_every,
 * 2 * sample_every, ... (sample_every 0 counts as 1) are sweep generations:
 * their main repair pass also runs under every candidate partitioning, back to
 * back, each one timed on the device; totals add up over the sweeps.  Streams
 * also cost host time and waits outside the pass, so CT_SCAN_STREAMS is decided
 * on whole generations: the generations between sweeps run in blocks of four
 * with the best candidate with and the best without streams, alternating,
 * timed by the host clock; the lower mean block time wins (with no room for
 * blocks, the lowest sweep total wins).  The repair load changes as the
 * populations converge, so sweeps spread over a run choose better than its
 * first generations alone.  Every candidate computes the same result, so the
 * runs' state advances exactly as with ct_batch_step.  The choice is kept for
 * the batch and, process-wide, for later batches of the same shape (per run:
 * algorithm, row bytes, parameters, log2 |V|, log2 P); when the shape was tuned
 * before and force is 0 these are plain generations.  Synchronises the stream
 * at each sweep and block.
 */
int ct_batch_autotune(ct_batch* b, uint32_t n_generations, uint32_t sample_every, uint32_t force, void* stream);
/*
 * ct_batch_set_tuning -- install a scan partitioning for this batch (one saved
 * from ct_batch_tuning, say): items in [64, 32768], min_boxes in [1, 2^20],
 * grid_waves in [64, 2^20], mode one of CT_SCAN_*; CT_EINVAL otherwise.
 * Results do not depend on it.  The batch counts as tuned; the process-wide
 * cache is left alone.  CT_SCAN_STREAMS on a batch of one run launches serially.
 */
int ct_batch_set_tuning(ct_batch* b, uint32_t items, uint32_t min_boxes, uint32_t grid_waves, uint32_t mode);
/* The batch's scan partitioning and whether it came from tuning. */
int ct_batch_tuning(const ct_batch* b, uint32_t* items, uint32_t* min_boxes, uint32_t* grid_waves,
                    uint32_t* mode, uint32_t* tuned);

/*
 * ct_pop_read -- copy a run's state to the host (synchronises its stream).
 * h_pos[pop_size]: population as valid-list positions (PSO: the personal-best
 * configurations; Firefly: each firefly's last evaluated configuration);
 * h_f[pop_size]: their objective values.  Any output may be
 * NULL.  *best_pos / *best_f: best configuration found so far.
 */
int ct_pop_read(const ct_pop* p, uint32_t* h_pos, float* h_f, uint32_t* best_pos, float* best_f,
                uint32_t* generation, uint32_t* reinits);

/*
 * ct_pop_evaluated -- the configurations the last generation evaluated (after creation: the
 * initial population), as valid-list positions, one per individual in individual order
 * (h_pos[pop_size]): DE's trials after repair, PSO's and Firefly's evaluated (repaired) positions,
 * GA's children after repair and mutation; 0xFFFFFFFF for an invalid configuration of a
 * non-aware run.  A DE generation that reinitialised its population (the reinits counter of
 * ct_pop_read went up) then evaluated the new members too: ct_pop_read's positions.
 * Synchronises.  After ct_pop_restore the output is undefined until the next generation.
 */
int ct_pop_evaluated(const ct_pop* p, uint32_t* h_pos);

/* Cumulative number of configurations the run has sent through a repair scan
   (invalid proposals) and through a mutation scan (GA).  Synchronises. */
int ct_pop_counters(const ct_pop* p, uint64_t* repairs, uint64_t* mutations);

/*
 * ct_pop_snapshot / ct_pop_restore -- full run state as bytes (synchronising).
 * Layout: uint32 header[8] = {magic 0x43545031 (non-aware runs: 0x43545531), algo,
 * pop_size, n_params, generation, reinits, best_pos, best_f bits}, then for DE/GA uint32
 * pos[P], float f[P] (non-aware: followed by uint8 rows[P][D], the members' digits); for
 * Firefly uint32 pos[P] (evaluated positions), float f[P] (brightness), int32 X[P][D]; for
 * PSO int32 X[P][D], int64 V[P][D], int32 PB[P][D], float f_pb[P], uint32 pb_pos[P],
 * uint32 gbest_index.  Call with h_buf = NULL to get the size.  A restored run continues
 * bit-identically.  ct_pop_restore checks the whole snapshot on the host before it writes
 * anything to the device: the run's shape (algorithm, pop_size, n_params, aware or not),
 * every position and best_pos below n_valid (non-aware runs: or 0xFFFFFFFF), aware DE
 * positions distinct, non-aware digits inside their domains, PSO and Firefly coordinates X
 * and PB in [0, M * 2^16) (M the largest radix), |V| < 2^46 and gbest_index < pop_size; on
 * CT_EINVAL the run is left as it was.
 */
int ct_pop_snapshot(const ct_pop* p, void* h_buf, size_t* len);
int ct_pop_restore(ct_pop* p, const void* h_buf, size_t len);

void ct_pop_free(ct_pop* p);

/*
 * Device bytes held by a built space (bitmask, valid list, rank directory,
 * bounding boxes, value tables) and by a run (population state and repair
 * scratch; DE adds 4 bytes + 1 bit per valid configuration).  Sizes are the
 * bytes requested from the allocator.  The objective table is the caller's.
 */
int ct_space_footprint(const ct_space* s, uint64_t* bytes);
int ct_pop_footprint(const ct_pop* p, uint64_t* bytes);

/*
 * Serving (many optimiser runs arriving over time on one GPU).
 *
 * A server keeps every admitted run's space, population and objective table
 * resident and advances all admitted runs together, one generation per
 * ct_server_step, as one batch (same kernels and results as ct_batch_step).
 * Runs are admitted in submission order when (a) fewer than max_active runs
 * are active and (b) the run's footprint -- its resolved space, its
 * population state and its objective table, in bytes as ct_space_footprint /
 * ct_pop_footprint count them -- fits in hbm_budget beside the active runs.
 * A run's space is resolved at admission on a second stream while the current
 * generation runs; the resolution stops before allocating the valid list if
 * it would not fit, and the run then waits.  Runs join and leave at generation
 * boundaries; each run's results equal those of stepping it alone.
 *
 * objective(ctx, run_id, n_valid, h_out) is called on the thread that calls
 * ct_server_step, once per admitted run, to fill h_out[n_valid] (float32 > 0,
 * indexed by valid-list position); a non-zero return ends the run with
 * CT_EINVAL.
 *
 * A population larger than the run's valid set is cut to n_valid (reported in
 * ct_run_result.pop_size).  A run that can never fit (footprint above
 * hbm_budget), has no valid configuration, or is DE with fewer than 4 valid
 * configurations ends with status CT_ENOMEM / CT_EEMPTY / CT_EINVAL instead
 * of running.  The server is not thread-safe:
 * one thread submits, steps and polls.
 */
typedef struct ct_server ct_server;
typedef int (*ct_objective_fn)(void* ctx, uint64_t run_id, uint64_t n_valid, float* h_out);

typedef struct {
    uint64_t hbm_budget;            /* bytes for resident runs */
    uint32_t max_active;            /* slot cap, 1..4096 */
    uint32_t max_admit_per_step;    /* 0 = no limit */
    uint32_t keep_snapshots;        /* keep each finished run's ct_pop_snapshot bytes */
    uint32_t reserved;
    ct_objective_fn objective;
    void* objective_ctx;
} ct_server_config;

typedef struct {
    uint64_t id;
    int32_t status;                 /* CT_OK, or why the run did not run */
    uint32_t generations;           /* generations completed */
    uint64_t n_valid;
    uint64_t footprint;             /* device bytes charged while resident */
    uint32_t best_pos;              /* best configuration (valid-list position) */
    float best_f;
    uint32_t reinits;
    uint32_t pop_size;
    double t_submit, t_admit, t_done;   /* seconds on the server clock; t_admit < 0: never admitted */
} ct_run_result;

typedef struct {
    uint64_t steps, run_generations, submitted, admitted, rejected, completed;
    uint64_t queued, active, used_bytes, peak_bytes;
} ct_server_counters;

int ct_server_create(const ct_server_config* cfg, ct_server** out);
/* Queue a run: the space (as for ct_space_build), its parameters and its
   generation count.  arrival_s < 0 stamps the submission with ct_server_now(). */
int ct_server_submit(ct_server* s, const int64_t* values, const uint32_t* radices, uint32_t n_params,
                     const uint32_t* code, const uint32_t* cons_offsets, uint32_t n_cons, const ct_pop_params* p,
                     uint32_t n_generations, double arrival_s, uint64_t* run_id);
/* One generation of the active runs (with admissions overlapped and
   retirements after it); *n_busy = active + queued runs afterwards. */
int ct_server_step(ct_server* s, uint32_t* n_busy);
double ct_server_now(const ct_server* s);
/* Finished runs not yet polled, oldest first (at most cap). */
int ct_server_poll(ct_server* s, ct_run_result* out, uint32_t cap, uint32_t* n_out);
/* The kept snapshot of a finished run (h_buf = NULL: size only). */
int ct_server_snapshot(const ct_server* s, uint64_t run_id, void* h_buf, size_t* len);
/* Drop a polled run's host record. */
int ct_server_release(ct_server* s, uint64_t run_id);
int ct_server_stats(const ct_server* s, ct_server_counters* out);
/* Step intervals: completion-to-completion milliseconds of consecutive
   generations and the number of runs each advanced (cap = 0: count only). */
int ct_server_step_times(const ct_server* s, float* h_ms, uint32_t* h_active, uint64_t cap, uint64_t* n_out);
void ct_server_free(ct_server* s);

/*
 * Kernel timing (measurement support, not part of the method).  While enabled,
 * the library records a pair of HIP events on the launch stream around every
 * kernel launch; ct_prof_read synchronises and returns the summed elapsed time
 * and the number of launches of the kernel with the given base name (for
 * example "k_repair_scan", "k_mask", "k_de_select").  Enabling or disabling
 * clears the records.
 */
int ct_prof_enable(int on);
int ct_prof_read(const char* kernel, double* total_ms, uint64_t* launches);
/* Record events only around launches of the named kernel (NULL: every kernel). */
int ct_prof_select(const char* kernel);
/* Record events only around every `every`-th launch of each kernel name (counted from the last
   ct_prof_enable; every = 1, the default: all of them; 0 is CT_EINVAL).  Each recorded event
   stalls the stream around its launch by a few microseconds, so sampling keeps the timed work
   close to unmeasured work while the sampled launches still give the mean launch time. */
int ct_prof_sample(uint32_t every);
/* Launches of the named kernel since the last ct_prof_enable that passed the ct_prof_select
   filter, recorded or not (with sampling, ct_prof_read counts only the recorded ones). */
int ct_prof_seen(const char* kernel, uint64_t* launches);
/* Repair scans of the main pass are "k_repair_scan", those of the Hamming fallback pass of
   Alg. 2/3 candidates without a tier 0-2 neighbour "k_repair_scan_fb".
   ct_prof_count_boxes(1) clears and starts device counters of the work the scans actually do:
   while on, every scan item adds the 64-row boxes whose rows it evaluated and the 64-box chunks
   it opened (outside graph capture and tuning sweeps); ct_prof_boxes (synchronising) returns
   {main-pass boxes, main-pass chunks, fallback boxes, fallback chunks}. */
int ct_prof_count_boxes(int on);
int ct_prof_boxes(uint64_t* out4);

#ifdef __cplusplus
}
#endif

#endif /* CT_H */
