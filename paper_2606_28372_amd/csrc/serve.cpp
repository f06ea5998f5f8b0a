// Serving loop: optimiser runs arrive over time, are admitted by their
// device-memory footprint (resolved space + population + objective table) and
// advance together in one continuously re-formed batch, one generation per
// server step.  Runs join and leave at generation boundaries; a run's results
// do not depend on which other runs shared its steps, because every random
// draw is named by (seed, individual, generation, purpose) and every kernel
// works on per-run state only.
//
// One server step:
//   1. launch one generation of every active run (the batch's descriptors were
//      refilled while the device was idle at the end of the previous step);
//   2. while it runs, admit queued runs in arrival order as long as the slot cap
//      and the byte budget allow: resolve the space on a second stream (under a
//      byte limit, so a space that turns out too large never allocates its
//      list), fill the objective table through the caller's callback, create
//      the run;
//   3. wait for the generation, record its completion event;
//   4. retire runs that reached their generation count (results to the host,
//      device memory released) and refill the batch for the next step.
// Step latency is the interval between consecutive completion events, so it
// includes every gap the host leaves between generations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "ct_host.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Run {
    uint64_t id = 0;
    ct_space* space = nullptr;      // host layout from submit; device parts while resident
    ct_pop_params prm{};
    uint32_t gens = 0, done = 0;
    float* d_obj = nullptr;
    ct_pop* pop = nullptr;
    uint64_t footprint = 0;         // exact device bytes once the valid-set size is known
    uint64_t n_valid = 0;
    bool sized = false;
    double t_submit = 0, t_admit = -1, t_done = -1;
    int status = CT_OK;
    uint32_t best_pos = 0, reinits = 0;
    float best_f = 0;
    std::vector<uint8_t> snap;
};

void release_space_device(ct_space* s) {
    void* bufs[] = {s->d_values, s->d_code, s->d_prefix, s->d_words, s->d_lin, s->d_rows, s->d_prevnext,
                    s->d_grp_off, s->d_dir8, s->d_boxes, s->d_dev};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    s->d_values = nullptr; s->d_code = nullptr; s->d_prefix = nullptr; s->d_words = nullptr;
    s->d_lin = nullptr; s->d_rows = nullptr; s->d_prevnext = nullptr; s->d_grp_off = nullptr;
    s->d_dir8 = nullptr; s->d_boxes = nullptr; s->d_dev = nullptr;
    s->dev_bytes = 0;
}

}  // namespace

struct ct_server {
    ct_server_config cfg{};
    hipStream_t st = nullptr;        // generations
    hipStream_t st_build = nullptr;  // admissions (space builds, run initialisation)
    Clock::time_point t0;
    uint64_t next_id = 1;
    std::deque<Run*> queue;
    std::vector<Run*> active;
    std::vector<Run*> unpolled;
    std::unordered_map<uint64_t, Run*> finished;
    ct_batch* batch = nullptr;
    bool dirty = true;
    uint64_t used = 0, peak = 0;
    hipEvent_t ev_last = nullptr;    // completion of the latest step, when it follows another step
    std::vector<hipEvent_t> ev_pool;
    std::vector<float> step_ms;
    std::vector<uint32_t> step_active;
    uint64_t steps = 0, run_generations = 0, submitted = 0, admitted = 0, rejected = 0, completed = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    void finish(Run* r, int status) {
        r->status = status;
        r->t_done = now();
        if (status != CT_OK) rejected++;
        else completed++;
        if (r->pop) { ct_pop_free(r->pop); r->pop = nullptr; }
        if (r->d_obj) { (void)hipFree(r->d_obj); r->d_obj = nullptr; }
        if (r->space) { ct_space_free(r->space); r->space = nullptr; }
        unpolled.push_back(r);
        finished[r->id] = r;
    }

    // bytes of a run with a resolved space of n_valid configurations
    uint64_t run_bytes(const Run* r, uint64_t n_valid) const {
        const ct_space* s = r->space;
        return space_resident_bytes(s, n_valid) +
               pop_footprint_bytes(r->prm.algo, r->prm.pop_size, s->D, s->R, n_valid, r->prm.unaware) +
               std::max<uint64_t>(n_valid, 1) * sizeof(float);
    }

    // Admit queued runs in arrival order; returns a HIP failure only (per-run failures end that run).
    int admit() {
        uint32_t n_admitted = 0;
        while (!queue.empty() && active.size() < cfg.max_active &&
               (cfg.max_admit_per_step == 0 || n_admitted < cfg.max_admit_per_step)) {
            Run* r = queue.front();
            const uint64_t avail = cfg.hbm_budget > used ? cfg.hbm_budget - used : 0;
            const uint64_t scratch = space_build_scratch_bytes(r->space);
            if (!r->sized) {
                const uint64_t floor_bytes = space_resident_bytes(r->space, 0) + scratch;
                if (floor_bytes > cfg.hbm_budget) { queue.pop_front(); finish(r, CT_ENOMEM); continue; }
                if (floor_bytes > avail) break;
            } else if (r->footprint + scratch > avail) {
                break;
            }
            // resolve the space; the byte limit stops it before it allocates a list that cannot fit
            const uint64_t limit = avail - scratch;
            int rc = space_realize(r->space, st_build, limit);
            const bool over = rc == CT_ENOMEM && r->space->over_limit;
            if (rc && !over) {
                release_space_device(r->space);
                queue.pop_front();
                finish(r, rc);
                continue;
            }
            r->n_valid = r->space->n_valid;
            // an aware sample is stratified over the valid list: at most one member per configuration
            if (!r->prm.unaware && r->prm.pop_size > r->n_valid) r->prm.pop_size = (uint32_t)r->n_valid;
            r->footprint = run_bytes(r, r->n_valid);
            r->sized = true;
            const bool unusable = r->n_valid == 0 || r->n_valid > CT_MAX_VALID ||
                                  (r->prm.algo == CT_DE && r->prm.pop_size < de_min_pop(r->prm.de_method));
            if (unusable || r->footprint + scratch > cfg.hbm_budget) {
                release_space_device(r->space);
                queue.pop_front();
                finish(r, r->n_valid == 0 ? CT_EEMPTY : unusable ? CT_EINVAL : CT_ENOMEM);
                continue;
            }
            if (over || used + r->footprint > cfg.hbm_budget) {
                // does not fit beside the active runs: wait (device memory released meanwhile)
                release_space_device(r->space);
                break;
            }
            // objective table through the caller
            std::vector<float> h(r->n_valid);
            if (!cfg.objective || cfg.objective(cfg.objective_ctx, r->id, r->n_valid, h.data()) != 0) {
                release_space_device(r->space);
                queue.pop_front();
                finish(r, CT_EINVAL);
                continue;
            }
            if (hipMalloc(&r->d_obj, r->n_valid * sizeof(float)) != hipSuccess) {
                release_space_device(r->space);
                queue.pop_front();
                finish(r, CT_ENOMEM);
                continue;
            }
            CT_HIP(hipMemcpyAsync(r->d_obj, h.data(), r->n_valid * sizeof(float), hipMemcpyHostToDevice, st_build));
            rc = ct_pop_create(r->space, &r->prm, r->d_obj, st_build, &r->pop);
            CT_HIP(hipStreamSynchronize(st_build));
            queue.pop_front();
            if (rc) {
                (void)hipFree(r->d_obj);
                r->d_obj = nullptr;
                finish(r, rc);
                continue;
            }
            used += r->footprint;
            peak = std::max(peak, used);
            r->t_admit = now();
            active.push_back(r);
            admitted++;
            n_admitted++;
            dirty = true;
        }
        return CT_OK;
    }

    int refill() {
        if (!dirty) return CT_OK;
        std::vector<ct_pop*> pops;
        for (Run* r : active) pops.push_back(r->pop);
        if (!batch) {
            int rc = batch_build(pops, &batch, st);
            if (rc) return rc;
        } else {
            int rc = batch_fill(batch, pops);
            if (rc) return rc;
        }
        dirty = false;
        return CT_OK;
    }

    int step(uint32_t* busy) {
        int rc = CT_OK;
        hipEvent_t ev = nullptr;
        std::vector<Run*> stepped;
        if (!active.empty()) {
            if ((rc = refill())) return rc;
            if ((rc = batch_generation(batch, st))) return rc;
            ev = take_event();
            if (!ev) return ct_fail(CT_EDEVICE, "ct_server_step: hipEventCreate failed");
            CT_HIP(hipEventRecord(ev, st));
            stepped = active;
            steps++;
            run_generations += active.size();
        }
        // admissions overlap the running generation
        if ((rc = admit())) return rc;
        if (ev) {
            CT_HIP(hipEventSynchronize(ev));
            if (ev_last) {
                float ms = 0;
                CT_HIP(hipEventElapsedTime(&ms, ev_last, ev));
                step_ms.push_back(ms);
                step_active.push_back((uint32_t)stepped.size());
                ev_pool.push_back(ev_last);
            }
            ev_last = ev;
            // retire the runs that reached their generation count
            // runs admitted during this step were appended after the ones it advanced
            std::vector<Run*> keep;
            for (size_t k = 0; k < active.size(); k++) {
                Run* r = active[k];
                if (k >= stepped.size()) { keep.push_back(r); continue; }
                r->done++;
                if (r->done < r->gens) { keep.push_back(r); continue; }
                size_t len = 0;
                if ((rc = ct_pop_read(r->pop, nullptr, nullptr, &r->best_pos, &r->best_f, nullptr, &r->reinits)))
                    return rc;
                if (cfg.keep_snapshots) {
                    if ((rc = ct_pop_snapshot(r->pop, nullptr, &len))) return rc;
                    r->snap.resize(len);
                    if ((rc = ct_pop_snapshot(r->pop, r->snap.data(), &len))) return rc;
                }
                used -= r->footprint;
                dirty = true;
                finish(r, CT_OK);
            }
            active.swap(keep);
            if (active.empty() && ev_last) {
                // idle: the next step's interval would include the idle time
                ev_pool.push_back(ev_last);
                ev_last = nullptr;
            }
        }
        if (busy) *busy = (uint32_t)(active.size() + queue.size());
        return CT_OK;
    }
};

extern "C" {

int ct_server_create(const ct_server_config* cfg, ct_server** out) {
    if (!cfg || !out) return ct_fail(CT_EINVAL, "ct_server_create: null argument");
    *out = nullptr;
    if (cfg->max_active < 1 || cfg->max_active > 4096)
        return ct_fail(CT_EINVAL, "ct_server_create: max_active must be 1..4096");
    if (!cfg->objective) return ct_fail(CT_EINVAL, "ct_server_create: objective callback required");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return ct_fail(CT_EDEVICE, "no HIP device available");
    ct_server* s = new ct_server();
    s->cfg = *cfg;
    s->t0 = Clock::now();
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->st_build, hipStreamNonBlocking) != hipSuccess) {
        ct_server_free(s);
        return ct_fail(CT_EDEVICE, "ct_server_create: hipStreamCreate failed");
    }
    *out = s;
    return CT_OK;
}

int ct_server_submit(ct_server* s, const int64_t* values, const uint32_t* radices, uint32_t n_params,
                     const uint32_t* code, const uint32_t* cons_offsets, uint32_t n_cons, const ct_pop_params* prm,
                     uint32_t n_generations, double arrival_s, uint64_t* run_id) {
    if (!s || !prm || !run_id) return ct_fail(CT_EINVAL, "ct_server_submit: null argument");
    if (n_generations < 1) return ct_fail(CT_EINVAL, "ct_server_submit: n_generations must be >= 1");
    if (prm->algo > CT_FIREFLY) return ct_fail(CT_EINVAL, "ct_server_submit: unknown algorithm");
    if ((prm->algo == CT_DE && (prm->de_method > CT_DE_RANDTOBEST1 || prm->de_crossover > CT_DE_EXP)) ||
        (prm->algo == CT_GA && prm->ga_crossover > CT_GA_DISRUPTIVE_UNIFORM))
        return ct_fail(CT_EINVAL, "ct_server_submit: unknown operator");
    if (prm->unaware > 1 || (prm->unaware && prm->algo == CT_DE && prm->pop_size > CT_UNAWARE_DE_MAX_POP))
        return ct_fail(CT_EINVAL, "ct_server_submit: unaware is 0 or 1 (non-aware DE: pop_size <= 8192)");
    ct_space* sp = nullptr;
    int rc = space_prepare(values, radices, n_params, code, cons_offsets, n_cons, &sp);
    if (rc) return rc;
    Run* r = new Run();
    r->id = s->next_id++;
    r->space = sp;
    r->prm = *prm;
    r->gens = n_generations;
    r->t_submit = arrival_s >= 0 ? arrival_s : s->now();
    s->queue.push_back(r);
    s->submitted++;
    *run_id = r->id;
    return CT_OK;
}

int ct_server_step(ct_server* s, uint32_t* n_busy) {
    if (!s) return ct_fail(CT_EINVAL, "ct_server_step: null server");
    return s->step(n_busy);
}

double ct_server_now(const ct_server* s) { return s ? s->now() : 0.0; }

int ct_server_poll(ct_server* s, ct_run_result* out, uint32_t cap, uint32_t* n_out) {
    if (!s || !n_out || (cap && !out)) return ct_fail(CT_EINVAL, "ct_server_poll: null argument");
    uint32_t n = 0;
    while (n < cap && !s->unpolled.empty()) {
        Run* r = s->unpolled.front();
        s->unpolled.erase(s->unpolled.begin());
        ct_run_result& o = out[n++];
        o.id = r->id;
        o.status = r->status;
        o.generations = r->done;
        o.n_valid = r->n_valid;
        o.footprint = r->footprint;
        o.best_pos = r->best_pos;
        o.best_f = r->best_f;
        o.reinits = r->reinits;
        o.pop_size = r->prm.pop_size;
        o.t_submit = r->t_submit;
        o.t_admit = r->t_admit;
        o.t_done = r->t_done;
    }
    *n_out = n;
    return CT_OK;
}

int ct_server_snapshot(const ct_server* s, uint64_t run_id, void* h_buf, size_t* len) {
    if (!s || !len) return ct_fail(CT_EINVAL, "ct_server_snapshot: null argument");
    auto it = s->finished.find(run_id);
    if (it == s->finished.end() || it->second->snap.empty())
        return ct_fail(CT_EINVAL, "ct_server_snapshot: no kept snapshot for this run");
    const std::vector<uint8_t>& v = it->second->snap;
    if (!h_buf) { *len = v.size(); return CT_OK; }
    if (*len < v.size()) return ct_fail(CT_EINVAL, "ct_server_snapshot: buffer too small");
    std::copy(v.begin(), v.end(), static_cast<uint8_t*>(h_buf));
    *len = v.size();
    return CT_OK;
}

int ct_server_release(ct_server* s, uint64_t run_id) {
    if (!s) return ct_fail(CT_EINVAL, "ct_server_release: null server");
    auto it = s->finished.find(run_id);
    if (it == s->finished.end()) return ct_fail(CT_EINVAL, "ct_server_release: unknown or unfinished run");
    for (size_t k = 0; k < s->unpolled.size(); k++)
        if (s->unpolled[k] == it->second) return ct_fail(CT_EINVAL, "ct_server_release: run not polled yet");
    delete it->second;
    s->finished.erase(it);
    return CT_OK;
}

int ct_server_stats(const ct_server* s, ct_server_counters* o) {
    if (!s || !o) return ct_fail(CT_EINVAL, "ct_server_stats: null argument");
    o->steps = s->steps;
    o->run_generations = s->run_generations;
    o->submitted = s->submitted;
    o->admitted = s->admitted;
    o->rejected = s->rejected;
    o->completed = s->completed;
    o->queued = s->queue.size();
    o->active = s->active.size();
    o->used_bytes = s->used;
    o->peak_bytes = s->peak;
    return CT_OK;
}

int ct_server_step_times(const ct_server* s, float* h_ms, uint32_t* h_active, uint64_t cap, uint64_t* n_out) {
    if (!s || !n_out) return ct_fail(CT_EINVAL, "ct_server_step_times: null argument");
    const uint64_t n = std::min<uint64_t>(cap, s->step_ms.size());
    if (n && (!h_ms || !h_active)) return ct_fail(CT_EINVAL, "ct_server_step_times: null output");
    std::copy(s->step_ms.begin(), s->step_ms.begin() + n, h_ms);
    std::copy(s->step_active.begin(), s->step_active.begin() + n, h_active);
    *n_out = cap ? n : s->step_ms.size();
    return CT_OK;
}

void ct_server_free(ct_server* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (Run* r : s->active) {
        if (r->pop) ct_pop_free(r->pop);
        if (r->d_obj) (void)hipFree(r->d_obj);
        if (r->space) ct_space_free(r->space);
        delete r;
    }
    for (Run* r : s->queue) {
        if (r->space) ct_space_free(r->space);
        delete r;
    }
    for (auto& kv : s->finished) delete kv.second;
    if (s->batch) batch_free(s->batch);
    if (s->ev_last) (void)hipEventDestroy(s->ev_last);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->st) (void)hipStreamDestroy(s->st);
    if (s->st_build) (void)hipStreamDestroy(s->st_build);
    delete s;
}

}  // extern "C"
