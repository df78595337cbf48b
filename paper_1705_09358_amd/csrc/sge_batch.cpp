// Batching: many (pattern, target) jobs of uneven size in one persistent
// launch captured in a HIP graph, with an autotuner that picks between one
// search unit per job and root chunks of every job shared by all units, and
// the unit width (lanes per unit).
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
    std::vector<InstanceSpec> specs(njobs);
    for (uint32_t i = 0; i < njobs; i++) {
        auto it = c->targets.find(jobs[i].target);
        if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "job " + std::to_string(i) + ": unknown target");
        auto ip = c->patterns.find(jobs[i].pattern);
        if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "job " + std::to_string(i) + ": unknown pattern");
        if (jobs[i].mode < SGE_RI || jobs[i].mode > SGE_RIDS_SI_FC)
            return fail(c, SGE_E_INVAL, "job " + std::to_string(i) + ": unknown mode");
        specs[i].t = it->second.get();
        specs[i].p = ip->second.get();
        specs[i].mode = jobs[i].mode;
        specs[i].labelled = jobs[i].labelled != 0;
    }
    std::vector<InstanceOut> out;
    double mp = 0, ms = 0;
    int policy = c->batch_policy;
    int saved_lanes = c->lanes;
    const int saved_donate = c->donate;
    if (policy == 0) {
        auto it = c->batch_tune.find(njobs);   // repeated runs of one workload reuse the choice
        if (it == c->batch_tune.end()) {
            // autotune on this batch: the default shape first (root chunks,
            // automatic width, default donation period), then one unit per job,
            // the two widest units and a shorter donation period.  Exploring
            // stops once a trial runs longer than TUNE_MAX_TRIAL_MS: long
            // launches keep the best shape tried so far.
            constexpr double TUNE_MAX_TRIAL_MS = 100.0;
            double best = 1e300;
            BatchTune choice{2, 0, saved_donate};
            const int lanes[3] = {0, 32, 64};
            const int policies[2] = {2, 1};
            const int periods[2] = {1, 16};   // 1 = the default period
            bool stop = false;
            for (int l : lanes)
                for (int d : periods)
                    for (int p : policies) {
                        if (stop) continue;
                        if (saved_lanes && l != 0) continue;      // a width set by the caller is kept
                        if (saved_donate != 1 && d != 1) continue; // so is a donation setting
                        c->lanes = saved_lanes ? saved_lanes : l;
                        c->donate = saved_donate != 1 ? saved_donate : d;
                        sge_status st = run_instances(c, specs, out, mp, ms, true, p);
                        if (st == SGE_OK && ms <= TUNE_MAX_TRIAL_MS) {   // short launches: the better of two
                            double ms2 = 0;
                            st = run_instances(c, specs, out, mp, ms2, true, p);
                            ms = std::min(ms, ms2);
                        }
                        c->lanes = saved_lanes;
                        c->donate = saved_donate;
                        if (st != SGE_OK) return st;
                        if (ms < best) { best = ms; choice = BatchTune{p, l, saved_donate != 1 ? saved_donate : d}; }
                        if (ms > TUNE_MAX_TRIAL_MS) stop = true;
                    }
            it = c->batch_tune.emplace(njobs, choice).first;
        }
        policy = it->second.policy;
        c->lanes = saved_lanes ? saved_lanes : it->second.lanes;
        c->donate = it->second.donate;
    }
    sge_status st = run_instances(c, specs, out, mp, ms, true, policy);
    c->lanes = saved_lanes;
    c->donate = saved_donate;
    if (st != SGE_OK) return st;
    bool aborted = false, timed_out = false;
    for (uint32_t i = 0; i < njobs; i++) {
        results[i].matches = out[i].matches;
        results[i].states = out[i].states;
        results[i].candidates = out[i].candidates;
        results[i].steals = out[i].steals;
        results[i].steps = out[i].steps;
        results[i].ms_prep = mp;
        results[i].ms_search = ms;
        aborted |= out[i].status == SGE_E_ABORTED;
        timed_out |= out[i].timed_out;
    }
    if (timed_out) return fail(c, SGE_E_ABORTED, "batch stopped at the time limit; counters are partial");
    if (aborted) return fail(c, SGE_E_ABORTED, "state cap exceeded by at least one job");
    return SGE_OK;
}

}  // extern "C"
