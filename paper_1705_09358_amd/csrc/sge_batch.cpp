// Batching: many (pattern, target) jobs of uneven size in one persistent
// launch captured in a HIP graph, with an autotuner that picks between one
// search unit per job and root chunks of every job shared by all units, the
// unit width (lanes per unit), the resident blocks per CU and the donation
// period.
#include <algorithm>
#include <chrono>

#include "sge_ctx.h"

using namespace sge;


extern "C" {

sge_status sge_set_batch_policy(sge_ctx *c, int policy) {
    if (!c) return SGE_E_INVAL;
    if (policy < 0 || policy > 2) return fail(c, SGE_E_INVAL, "batch policy must be 0, 1 or 2");
    c->batch_policy = policy;
    return SGE_OK;
}

sge_status sge_batch_run(sge_ctx *c, uint32_t njobs, const sge_job *jobs, sge_result *results) {
    if (!c || (njobs && (!jobs || !results))) return SGE_E_INVAL;
    (void)hipSetDevice(c->device);
    std::vector<InstanceSpec> job_specs(njobs);
    for (uint32_t i = 0; i < njobs; i++) {
        auto it = c->targets.find(jobs[i].target);
        if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "job " + std::to_string(i) + ": unknown target");
        auto ip = c->patterns.find(jobs[i].pattern);
        if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "job " + std::to_string(i) + ": unknown pattern");
        if (jobs[i].mode < SGE_RI || jobs[i].mode > SGE_RIDS_SI_FC)
            return fail(c, SGE_E_INVAL, "job " + std::to_string(i) + ": unknown mode");
        job_specs[i].t = it->second.get();
        job_specs[i].p = ip->second.get();
        job_specs[i].mode = jobs[i].mode;
        job_specs[i].labelled = jobs[i].labelled != 0;
    }
    std::vector<InstanceSpec> specs = job_specs;   // in launch order
    std::vector<InstanceOut> out;
    double mp = 0, ms = 0;
    int policy = c->batch_policy;
    const int saved_lanes = c->lanes, saved_donate = c->donate, saved_per_cu = c->per_cu;
    // repeated runs of one batch (the same jobs) reuse the autotuner's choice
    // and the steps each job took last time
    uint64_t key = 1469598103934665603ull;   // a multiplicative hash of the job list, word by word
    auto mix = [&](uint64_t v) {
        key = (key ^ v) * 0x9E3779B97F4A7C15ull;
        key ^= key >> 29;
    };
    mix(njobs);
    for (uint32_t i = 0; i < njobs; i++) {
        mix(jobs[i].target);
        mix(jobs[i].pattern);
        mix(((uint64_t)(uint32_t)jobs[i].mode << 1) | (jobs[i].labelled ? 1u : 0u));
    }
    // Longest first: root chunks are claimed in the order of the launch's
    // instances, so an expensive instance late in the list starts late and
    // finishes alone.  Once a job list has run, its next launches order the
    // instances by the steps each took last time, most first (the first
    // launch keeps the caller's order); results go back to job order.
    std::vector<uint32_t> perm(njobs);
    for (uint32_t i = 0; i < njobs; i++) perm[i] = i;
    auto apply_order = [&](const std::vector<uint64_t> &steps) {
        order_by_desc(steps.data(), njobs, perm.data());
        for (uint32_t i = 0; i < njobs; i++) specs[i] = job_specs[perm[i]];
    };
    auto record_steps = [&](const std::vector<InstanceOut> &o) {
        std::vector<uint64_t> &steps = c->batch_steps[key];
        steps.assign(njobs, 0);
        for (uint32_t i = 0; i < njobs; i++) steps[perm[i]] = o[i].steps;
    };
    if (c->batch_steps.size() >= 256) c->batch_steps.clear();
    {
        auto hs = c->batch_steps.find(key);
        if (hs != c->batch_steps.end() && hs->second.size() == njobs) apply_order(hs->second);
    }
    if (policy == 0) {
        auto it = c->batch_tune.find(key);
        if (it == c->batch_tune.end()) {
            // autotune on this batch, starting from the default shape (root
            // chunks, automatic width, default donation period, all resident
            // blocks): resident blocks per CU, then the unit width
            // and the donation period together, then one unit per job.  A knob
            // the caller set is kept.  A short launch is run once more and then
            // timed three times (the median counts); a shape already timed (the
            // automatic width is one of the explicit ones) is not timed again.
            // Launch times of one shape spread by several percent, so the best
            // of several medians is biased low: the two fastest shapes are
            // then timed again in alternation, five launches each, and the
            // lower median decides.  Exploring stops once a trial runs longer
            // than TUNE_MAX_TRIAL_MS, and long launches keep the best shape so
            // far without the final comparison.
            constexpr double TUNE_MAX_TRIAL_MS = 100.0;
            constexpr int FINAL_RUNS = 5;
            struct Tried {
                BatchTune t;
                double ms;
            };
            std::vector<Tried> tried;
            auto same = [](const BatchTune &a, const BatchTune &b) {
                return a.policy == b.policy && a.lanes == b.lanes && a.donate == b.donate && a.per_cu == b.per_cu;
            };
            auto timed_before = [&](const BatchTune &t) {
                for (const Tried &x : tried)
                    if (same(x.t, t)) return true;
                return false;
            };
            auto set_shape = [&](const BatchTune &t) {
                c->lanes = t.lanes;
                c->donate = t.donate;
                c->per_cu = t.per_cu;
            };
            auto restore_shape = [&]() {
                c->lanes = saved_lanes;
                c->donate = saved_donate;
                c->per_cu = saved_per_cu;
            };
            double best = 1e300;
            BatchTune cur{2, saved_lanes, saved_donate, saved_per_cu};
            bool stop = false;
            bool ordered_now = c->batch_steps.count(key) != 0;
            auto trial = [&](BatchTune t) -> sge_status {
                if (stop || (t.lanes && timed_before(t))) return SGE_OK;
                set_shape(t);
                sge_status st = run_instances(c, specs, out, mp, ms, true, t.policy);
                if (st == SGE_OK && !ordered_now) {
                    // the trials time the order later launches will use
                    record_steps(out);
                    apply_order(c->batch_steps[key]);
                    ordered_now = true;
                    st = run_instances(c, specs, out, mp, ms, true, t.policy);
                }
                if (t.lanes == 0) t.lanes = c->last_lanes;   // the width the automatic choice resolved to
                if (st == SGE_OK && timed_before(t)) {
                    restore_shape();
                    return SGE_OK;
                }
                if (st == SGE_OK && ms <= TUNE_MAX_TRIAL_MS) {
                    double r[3] = {0, 0, 0};
                    for (int i = 0; i < 3 && st == SGE_OK; i++) st = run_instances(c, specs, out, mp, r[i], true, t.policy);
                    std::sort(r, r + 3);
                    ms = r[1];
                }
                restore_shape();
                if (st != SGE_OK) return st;
                tried.push_back({t, ms});
                if (ms < best) {
                    best = ms;
                    cur = t;
                }
                if (ms > TUNE_MAX_TRIAL_MS) stop = true;
                return SGE_OK;
            };
            sge_status st = trial(cur);
            if (st == SGE_OK && saved_per_cu == 0)
                for (int b : {1, 2, 3})
                    if (st == SGE_OK) st = trial(BatchTune{cur.policy, cur.lanes, cur.donate, b});
            const BatchTune after_blocks = cur;
            // the unit width and the donation period interact (narrow units
            // gain more from a shorter period; many mid-sized instances from a
            // longer one, which gives fewer and larger tasks away), so they
            // are tried together
            const std::vector<int> widths = saved_lanes ? std::vector<int>{saved_lanes} : std::vector<int>{32, 64};
            const std::vector<int> periods = saved_donate == 1 ? std::vector<int>{1, 16, 64, 128} : std::vector<int>{saved_donate};
            for (int l : widths)
                for (int dn : periods)
                    if (st == SGE_OK) st = trial(BatchTune{after_blocks.policy, l, dn, after_blocks.per_cu});
            if (st == SGE_OK) st = trial(BatchTune{1, cur.lanes, cur.donate, cur.per_cu});
            if (st == SGE_OK && !stop && tried.size() >= 2) {
                std::sort(tried.begin(), tried.end(), [](const Tried &a, const Tried &b) { return a.ms < b.ms; });
                const BatchTune A = tried[0].t, B = tried[1].t;
                double ra[FINAL_RUNS], rb[FINAL_RUNS];
                for (int i = 0; i < FINAL_RUNS && st == SGE_OK; i++) {
                    set_shape(A);
                    st = run_instances(c, specs, out, mp, ra[i], true, A.policy);
                    if (st != SGE_OK) break;
                    set_shape(B);
                    st = run_instances(c, specs, out, mp, rb[i], true, B.policy);
                }
                restore_shape();
                if (st == SGE_OK) {
                    std::sort(ra, ra + FINAL_RUNS);
                    std::sort(rb, rb + FINAL_RUNS);
                    cur = rb[FINAL_RUNS / 2] < ra[FINAL_RUNS / 2] ? B : A;
                }
            }
            if (st != SGE_OK) return st;
            if (c->batch_tune.size() >= 256) c->batch_tune.clear();
            it = c->batch_tune.emplace(key, cur).first;
        }
        policy = it->second.policy;
        c->lanes = it->second.lanes;
        c->donate = it->second.donate;
        c->per_cu = it->second.per_cu;
    }
    sge_status st = run_instances(c, specs, out, mp, ms, true, policy);
    c->lanes = saved_lanes;
    c->donate = saved_donate;
    c->per_cu = saved_per_cu;
    if (st != SGE_OK) return st;
    record_steps(out);
    bool aborted = false, timed_out = false;
    for (uint32_t i = 0; i < njobs; i++) {
        sge_result &r = results[perm[i]];
        r.matches = out[i].matches;
        r.states = out[i].states;
        r.candidates = out[i].candidates;
        r.alg_bytes = out[i].bytes;
        r.steals = out[i].steals;
        r.steps = out[i].steps;
        r.ms_prep = mp;
        r.ms_search = ms;
        aborted |= out[i].status == SGE_E_ABORTED;
        timed_out |= out[i].timed_out;
    }
    if (timed_out) return fail(c, SGE_E_ABORTED, "batch stopped at the time limit; counters are partial");
    if (aborted) return fail(c, SGE_E_ABORTED, "state cap exceeded by at least one job");
    return SGE_OK;
}

}  // extern "C"
