// Serving loop of the TIMEST GPU library: resident graphs, a weight-set
// cache bounded by a device-memory budget, admission by footprint, and
// continuous batching of sample ranges across queries.
//
// Two threads own the device work, each with its own stream: the builder
// makes weight sets (one at a time, smallest first, each once its footprint
// fits the budget after evicting idle sets) and the sampler runs batched
// passes over every admitted query.  Weight builds therefore overlap the
// sampling of queries already admitted.  All shared state sits under one
// mutex; no device work runs while it is held.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tm_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct CacheEntry {
    tm_weights* w = nullptr;
    u64 bytes = 0;
    int refs = 0;      // admitted queries using it
    u64 last_use = 0;  // release counter at the last release
};

struct Query {
    u64 ticket = 0;
    int gid = 0;
    tm_graph* g = nullptr;
    HostPlan plan;
    u64 k = 0, seed = 0;
    std::string key;      // weight-set identity
    u64 est_bytes = 0;    // 64-bit footprint of its weight set
    u64 extra_bytes = 0;  // build temporaries on top of it
    Clock::time_point t_submit, t_admit;
    bool waited = false;  // found the budget full at least once
    bool wide = false;    // its set needs 128 bits (reserve and build that)
    int64_t nq = 0;       // intervals of its set
    CacheEntry* ce = nullptr;
    u64 next = 0;  // next sample id to draw
    JobSums sums;
    uint32_t passes = 0;
    uint32_t hit = 0;
};

struct Done {
    tm_result r;
    tm_query_info info;
    std::string msg;
};

// Identity of a weight set: graph, motif edges, delta and time order, tree edges and center.
std::string set_key(int gid, const HostPlan& P) {
    std::string k;
    auto put = [&k](int64_t v) { k.append(reinterpret_cast<const char*>(&v), sizeof v); };
    put(gid);
    put(P.mo.k);
    put(P.mo.l);
    put(P.mo.delta);
    for (int e = 0; e < P.mo.l; ++e) {
        put(P.mo.src[e]);
        put(P.mo.dst[e]);
    }
    put(P.tree.center);
    for (int e = 0; e < P.tree.n_edges; ++e) put(P.tree.edge[e]);
    // a partial order changes the tree's windows and the completions
    put(P.po);
    for (int e = 0; P.po && e < P.mo.l; ++e) put(P.mo.before[e]);
    return k;
}

using QueryPtr = std::unique_ptr<Query>;

}  // namespace

struct tm_server {
    // configuration
    u64 budget = 0, reserve = 0;
    u64 pass_samples = 0, job_chunk = 0;
    int max_jobs = 0;
    bool fifo = false;
    int device = 0;
    tm_allocator alloc{};        // the caller's allocator (has_alloc) of weight sets and passes
    bool has_alloc = false;
    hipStream_t st = nullptr;   // sampling passes
    hipStream_t bst = nullptr;  // weight builds

    // shared state (mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_build, cv_done, cv_idle;
    bool stop = false;
    bool building = false;  // the builder is inside a weight build (cv_idle when it leaves)
    std::vector<tm_graph*> graphs;
    std::deque<QueryPtr> arrivals;  // submitted, not yet looked up
    std::deque<QueryPtr> builds;    // waiting for their weight set
    std::deque<QueryPtr> ready;     // admitted by the builder, not yet sampling
    std::map<std::string, CacheEntry> cache;
    // sets found to need 128 bits: their later builds reserve (and build) 128
    std::set<std::string> wide_keys;
    u64 resident = 0;
    u64 releases = 0;
    std::unordered_map<u64, Done> done;
    std::unordered_map<u64, bool> live;  // submitted and not yet collected
    u64 next_ticket = 1;
    tm_server_stats stats{};

    // sampler-private
    std::vector<QueryPtr> active;

    std::thread sampler, builder;

    void run_sampler();
    void run_builder();
    bool make_room_locked(u64 need);
    void admit_locked(Query& q, CacheEntry& ce, bool hit);
    void pass();
    void finish(QueryPtr q, int status, const char* msg);
};

// Evict idle weight sets, least recently released first, until need more
// bytes fit the budget; false if they cannot.
bool tm_server::make_room_locked(u64 need) {
    const u64 cap = budget - reserve;
    while (resident + need > cap) {
        auto victim = cache.end();
        for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->second.refs == 0 &&
                (victim == cache.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == cache.end()) return false;
        resident -= victim->second.bytes;
        // idle: every pass that used it has completed on its stream
        tm_weights_destroy(victim->second.w);
        cache.erase(victim);
        ++stats.evictions;
        stats.resident_bytes = resident;
        stats.cached_sets = cache.size();
    }
    return true;
}

void tm_server::admit_locked(Query& q, CacheEntry& ce, bool hit) {
    q.ce = &ce;
    ++ce.refs;
    q.hit = hit ? 1 : 0;
    q.t_admit = Clock::now();
    if (hit) ++stats.weight_hits;
}

void tm_server::finish(QueryPtr q, int status, const char* msg) {
    Done d;
    std::memset(&d.r, 0, sizeof d.r);
    std::memset(&d.info, 0, sizeof d.info);
    d.r.k = q->k;
    if (q->ce) {
        const tm_weights* w = q->ce->w;
        d.r.q = w->q;
        d.r.W.lo = (u64)w->W;
        d.r.W.hi = (u64)(w->W >> 64);
        if (w->wide) d.r.flags |= TM_F_WIDE;
        if (w->W == 0) d.r.flags |= TM_F_W_ZERO;
    }
    if (status == TM_OK) {
        sums_to_result(q->sums, &d.r);
        if (d.r.status == TM_OK) finish_result(&d.r);
        status = d.r.status;
    }
    d.r.status = status;
    const Clock::time_point now = Clock::now();
    d.info.latency_ms = ms_between(q->t_submit, now);
    d.info.queued_ms = q->ce ? ms_between(q->t_submit, q->t_admit) : d.info.latency_ms;
    d.info.weights_hit = q->hit;
    d.info.passes = q->passes;
    if (status != TM_OK && msg) d.msg = msg;
    std::lock_guard<std::mutex> lk(mu);
    if (q->ce) {
        q->ce->last_use = ++releases;
        if (--q->ce->refs == 0) cv_build.notify_one();
    }
    if (status == TM_OK) ++stats.completed;
    else ++stats.failed;
    done[q->ticket] = std::move(d);
    cv_done.notify_all();
}

void tm_server::run_builder() {
    AllocScope scope_(has_alloc ? &alloc : nullptr);
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        // queries whose set is resident by now are admitted at once
        for (auto it = builds.begin(); it != builds.end();) {
            auto c = cache.find((*it)->key);
            if (c == cache.end()) {
                ++it;
                continue;
            }
            admit_locked(**it, c->second, true);
            ready.push_back(std::move(*it));
            it = builds.erase(it);
            cv_work.notify_one();
        }
        if (builds.empty()) {
            cv_build.wait(lk);
            continue;
        }
        // smallest set first (arrival order among equals)
        auto pick = builds.begin();
        for (auto it = builds.begin(); it != builds.end(); ++it)
            if ((*it)->est_bytes < (*pick)->est_bytes) pick = it;
        Query& q = **pick;
        if (!make_room_locked(q.est_bytes + q.extra_bytes)) {
            if (!q.waited) {
                q.waited = true;
                ++stats.admission_waits;
            }
            cv_build.wait(lk);  // a release or an arrival
            continue;
        }
        QueryPtr qp = std::move(*pick);
        builds.erase(pick);
        resident += qp->est_bytes + qp->extra_bytes;  // held while building
        building = true;
        lk.unlock();

        tm_weights* w = new (std::nothrow) tm_weights();
        int rc = w ? TM_OK : tm_fail(TM_ENOMEM, "server: host allocation");
        const Clock::time_point tb = Clock::now();
        if (w) {
            w->g = qp->g;
            w->arena.stream = bst;
            w->plan = qp->plan;
            // resident sets matter more here than the sampler's speed-up
            w->lean = true;
            // the budget is a hard bound: a build stays within what it
            // reserved, so a 64-bit build that needs 128 bits stops and the
            // query comes back with the 128-bit reservation
            w->width_mode = qp->wide ? 2 : 1;
            rc = weights_build(w, bst);
            if (rc == TM_ENOMEM) {
                // the device holds more than the budget counts (cached
                // blocks, other users): drop idle sets and cached blocks
                {
                    std::lock_guard<std::mutex> g(mu);
                    (void)make_room_locked(~(u64)0 >> 1);
                }
                dev_cache_trim();
                rc = weights_build(w, bst);
            }
        }
        const bool needs_wide = w && w->needs_wide;
        if (needs_wide) {
            // the 64-bit blocks go back to the block cache, which serves the
            // larger build from them where sizes allow (and returns cached
            // blocks to HIP by itself when an allocation fails)
            tm_weights_destroy(w);
            w = nullptr;
        }
        const std::string err = rc != TM_OK ? tm_last_error() : "";
        lk.lock();
        building = false;
        cv_idle.notify_all();
        resident -= qp->est_bytes + qp->extra_bytes;
        if (needs_wide) {
            wide_keys.insert(qp->key);
            qp->wide = true;
            qp->est_bytes = weights_footprint(qp->plan, qp->g->m, qp->nq, true, true);
            qp->extra_bytes = weights_build_extra(qp->g->m, true);
            if (qp->est_bytes + qp->extra_bytes > budget - reserve) {
                lk.unlock();
                finish(std::move(qp), TM_EADMIT, "server: the 128-bit weight set exceeds the budget");
                lk.lock();
            } else {
                // its other queries reserve the 128-bit size too
                for (auto& b : builds)
                    if (b->key == qp->key && !b->wide) {
                        b->wide = true;
                        b->est_bytes = qp->est_bytes;
                        b->extra_bytes = qp->extra_bytes;
                    }
                builds.push_front(std::move(qp));
            }
            continue;
        }
        if (rc == TM_ENOMEM) {
            tm_weights_destroy(w);
            bool pinned = false;
            for (auto& kv : cache) pinned |= kv.second.refs > 0;
            if (pinned) {
                // wait for running queries to release their sets
                if (!qp->waited) {
                    qp->waited = true;
                    ++stats.admission_waits;
                }
                builds.push_front(std::move(qp));
                cv_build.wait(lk);
                continue;
            }
        }
        if (rc != TM_OK) {
            if (rc != TM_ENOMEM) tm_weights_destroy(w);
            const std::string msg = err.empty() ? tm_last_error() : err;
            lk.unlock();
            finish(std::move(qp), rc, msg.c_str());
            lk.lock();
            continue;
        }
        // the set takes what its reservation held (the footprint is exact)
        if (resident + w->arena.bytes > budget - reserve && !make_room_locked(w->arena.bytes)) {
            tm_weights_destroy(w);
            if (!qp->waited) {
                qp->waited = true;
                ++stats.admission_waits;
            }
            builds.push_front(std::move(qp));
            cv_build.wait(lk);
            continue;
        }
        CacheEntry& ce = cache[qp->key];
        ce.w = w;
        ce.bytes = w->arena.bytes;
        ce.refs = 0;
        ce.last_use = releases;
        resident += ce.bytes;
        ++stats.weight_builds;
        stats.build_ms += ms_between(tb, Clock::now());
        stats.resident_bytes = resident;
        stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, resident + reserve);
        stats.cached_sets = cache.size();
        admit_locked(*qp, ce, false);
        ready.push_back(std::move(qp));
        cv_work.notify_one();
    }
}

void tm_server::pass() {
    // queries with nothing left to draw (k = 0, or W = 0) finish now
    for (size_t i = 0; i < active.size();) {
        Query& q = *active[i];
        if (q.next >= q.k || q.ce->w->W == 0) {
            QueryPtr qq = std::move(active[i]);
            active.erase(active.begin() + i);
            finish(std::move(qq), TM_OK, nullptr);
        } else {
            ++i;
        }
    }
    if (active.empty()) return;
    std::vector<Query*> order;
    for (auto& q : active) order.push_back(q.get());
    if (!fifo)
        std::stable_sort(order.begin(), order.end(),
                         [](const Query* a, const Query* b) { return a->k - a->next < b->k - b->next; });
    std::vector<Query*> pick;
    std::vector<tm_weights*> ws;
    std::vector<u64> j0, cnt, seeds;
    u64 taken = 0;
    for (Query* q : order) {
        if ((int)pick.size() >= max_jobs || taken >= pass_samples) break;
        const u64 c = std::min({q->k - q->next, job_chunk, pass_samples - taken});
        pick.push_back(q);
        ws.push_back(q->ce->w);
        j0.push_back(q->next);
        cnt.push_back(c);
        seeds.push_back(q->seed);
        taken += c;
    }
    std::vector<JobSums> sums(pick.size());
    const Clock::time_point tp = Clock::now();
    int rc = batch_sample_pass(ws.data(), j0.data(), cnt.data(), seeds.data(), (int)pick.size(), st, sums.data(),
                               batch_config_now());
    if (rc == TM_ENOMEM) {
        // the device held more than the budget counts (a build's temporaries
        // beyond its estimate, as in a 128-bit rebuild, or cached blocks):
        // wait for the build in flight, give the cached blocks back and run
        // the same pass once more
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_idle.wait(lk, [&] { return !building || stop; });
        }
        dev_cache_trim();
        sums.assign(pick.size(), JobSums{});
        rc = batch_sample_pass(ws.data(), j0.data(), cnt.data(), seeds.data(), (int)pick.size(), st, sums.data(),
                               batch_config_now());
        std::lock_guard<std::mutex> lk(mu);
        ++stats.pass_retries;
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        ++stats.passes;
        stats.samples += taken;
        stats.pass_ms += ms_between(tp, Clock::now());
    }
    for (size_t x = 0; x < pick.size(); ++x) {
        Query* q = pick[x];
        if (rc != TM_OK) q->sums.status = rc;
        else sums_merge(q->sums, sums[x]);
        q->next += cnt[x];
        ++q->passes;
    }
    const std::string err = rc != TM_OK ? tm_last_error() : "";
    for (size_t i = 0; i < active.size();) {
        Query& q = *active[i];
        const bool failed = q.sums.status != TM_OK || (q.sums.flags & 1);
        if (q.next >= q.k || failed) {
            QueryPtr qq = std::move(active[i]);
            active.erase(active.begin() + i);
            const int sq = qq->sums.status;
            finish(std::move(qq), sq, err.empty() ? nullptr : err.c_str());
        } else {
            ++i;
        }
    }
}

void tm_server::run_sampler() {
    AllocScope scope_(has_alloc ? &alloc : nullptr);
    (void)hipSetDevice(device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !arrivals.empty() || !ready.empty() || !active.empty(); });
            if (stop) break;
            bool to_build = false;
            while (!arrivals.empty()) {
                QueryPtr q = std::move(arrivals.front());
                arrivals.pop_front();
                auto c = cache.find(q->key);
                if (c != cache.end()) {
                    admit_locked(*q, c->second, true);
                    active.push_back(std::move(q));
                } else {
                    builds.push_back(std::move(q));
                    to_build = true;
                }
            }
            while (!ready.empty()) {
                active.push_back(std::move(ready.front()));
                ready.pop_front();
            }
            if (to_build) cv_build.notify_one();
        }
        if (!active.empty()) pass();
    }
}

extern "C" int tm_server_create(uint64_t budget_bytes, const tm_server_opts* opts, const tm_allocator* alloc,
                                tm_server** out) {
    if (!out) return tm_fail(TM_EINVAL, "server: NULL output");
    if (alloc && (!alloc->alloc || !alloc->free)) return tm_fail(TM_EINVAL, "server: allocator without alloc or free");
    std::unique_ptr<tm_server> s(new (std::nothrow) tm_server());
    if (!s) return tm_fail(TM_ENOMEM, "server: host allocation");
    if (alloc) {
        s->alloc = *alloc;
        s->has_alloc = true;
    }
    s->pass_samples = opts && opts->pass_samples ? opts->pass_samples : ((u64)1 << 24);
    s->job_chunk = opts && opts->job_chunk ? opts->job_chunk : ((u64)1 << 22);
    s->max_jobs = opts && opts->max_jobs > 0 ? opts->max_jobs : 256;
    s->fifo = opts && opts->fifo;
    if (s->pass_samples >= ((u64)1 << 31) || s->job_chunk > s->pass_samples)
        return tm_fail(TM_EINVAL, "server: pass_samples %llu, job_chunk %llu",
                       (unsigned long long)s->pass_samples, (unsigned long long)s->job_chunk);
    s->reserve = 24 * s->pass_samples;
    if (budget_bytes <= s->reserve)
        return tm_fail(TM_EINVAL, "server: budget %llu bytes below the pass reserve %llu",
                       (unsigned long long)budget_bytes, (unsigned long long)s->reserve);
    s->budget = budget_bytes;
    s->stats.budget_bytes = budget_bytes;
    TM_HIP(hipGetDevice(&s->device));
    TM_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    if (hipStreamCreateWithFlags(&s->bst, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->st);
        return tm_fail(TM_EDEVICE, "server: cannot create a stream");
    }
    tm_server* raw = s.get();
    try {
        s->sampler = std::thread([raw] { raw->run_sampler(); });
        s->builder = std::thread([raw] { raw->run_builder(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->cv_build.notify_all();
        if (s->sampler.joinable()) s->sampler.join();
        (void)hipStreamDestroy(s->st);
        (void)hipStreamDestroy(s->bst);
        return tm_fail(TM_EDEVICE, "server: cannot start its threads");
    }
    *out = s.release();
    return TM_OK;
}

extern "C" int tm_server_add_graph(tm_server* srv, tm_graph* g, int32_t* gid) {
    if (!srv || !g || !gid) return tm_fail(TM_EINVAL, "server_add_graph: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->graphs.push_back(g);
    *gid = (int32_t)srv->graphs.size() - 1;
    return TM_OK;
}

extern "C" int tm_server_submit(tm_server* srv, int32_t gid, const tm_motif* mo, const tm_tree* tr,
                                uint64_t k, uint64_t seed, uint64_t* ticket) {
    if (!srv || !ticket) return tm_fail(TM_EINVAL, "server_submit: NULL argument");
    tm_graph* g = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (gid < 0 || gid >= (int32_t)srv->graphs.size())
            return tm_fail(TM_EINVAL, "server_submit: unknown graph %d", gid);
        g = srv->graphs[gid];
    }
    TM_TRY(motif_check(mo));
    tm_tree def;
    if (!tr) {
        TM_TRY(tm_default_tree(mo, &def));
        tr = &def;
    }
    QueryPtr q(new (std::nothrow) Query());
    if (!q) return tm_fail(TM_ENOMEM, "server_submit: host allocation");
    TM_TRY(plan_build(mo, tr, &q->plan));
    if (g->m > 0 && g->T / mo->delta + 1 >= ((int64_t)1 << 31))
        return tm_fail(TM_ERANGE, "server_submit: too many intervals");
    const int64_t nq = g->m > 0 ? g->T / mo->delta + 1 : 0;
    q->nq = nq;
    q->key = set_key(gid, q->plan);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        q->wide = srv->wide_keys.count(q->key) != 0;
    }
    q->est_bytes = weights_footprint(q->plan, g->m, nq, q->wide, true);
    q->extra_bytes = weights_build_extra(g->m, q->wide);
    if (q->est_bytes + q->extra_bytes > srv->budget - srv->reserve)
        return tm_fail(TM_EADMIT, "server_submit: weight set of %llu bytes (+%llu while built), budget %llu",
                       (unsigned long long)q->est_bytes, (unsigned long long)q->extra_bytes,
                       (unsigned long long)(srv->budget - srv->reserve));
    q->gid = gid;
    q->g = g;
    q->k = k;
    q->seed = seed;
    q->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return tm_fail(TM_ECANCELED, "server_submit: server stopping");
        q->ticket = srv->next_ticket++;
        *ticket = q->ticket;
        srv->live[q->ticket] = true;
        ++srv->stats.submitted;
        srv->arrivals.push_back(std::move(q));
    }
    srv->cv_work.notify_one();
    return TM_OK;
}

static int collect(tm_server* srv, uint64_t ticket, tm_result* out, tm_query_info* info, bool block) {
    if (!srv) return tm_fail(TM_EINVAL, "server: NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->live.count(ticket))
        return tm_fail(TM_EINVAL, "server: unknown ticket %llu", (unsigned long long)ticket);
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) {
        if (!block) return TM_EAGAIN;
        srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) > 0; });
        it = srv->done.find(ticket);
    }
    Done d = std::move(it->second);
    srv->done.erase(it);
    srv->live.erase(ticket);
    lk.unlock();
    if (out) *out = d.r;
    if (info) *info = d.info;
    if (d.r.status != TM_OK)
        return tm_fail(d.r.status, "%s", d.msg.empty() ? tm_strerror(d.r.status) : d.msg.c_str());
    return TM_OK;
}

extern "C" int tm_server_poll(tm_server* srv, uint64_t ticket, tm_result* out, tm_query_info* info) {
    return collect(srv, ticket, out, info, false);
}

extern "C" int tm_server_wait(tm_server* srv, uint64_t ticket, tm_result* out, tm_query_info* info) {
    return collect(srv, ticket, out, info, true);
}

extern "C" int tm_server_read_stats(tm_server* srv, tm_server_stats* out) {
    if (!srv || !out) return tm_fail(TM_EINVAL, "server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    return TM_OK;
}

extern "C" void tm_server_destroy(tm_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    srv->cv_build.notify_all();
    srv->cv_idle.notify_all();
    if (srv->builder.joinable()) srv->builder.join();
    if (srv->sampler.joinable()) srv->sampler.join();
    // everything unfinished is cancelled
    std::vector<QueryPtr> rest;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto* dq : {&srv->arrivals, &srv->builds, &srv->ready})
            for (auto& q : *dq) rest.push_back(std::move(q));
        srv->arrivals.clear();
        srv->builds.clear();
        srv->ready.clear();
    }
    for (auto& q : srv->active) rest.push_back(std::move(q));
    srv->active.clear();
    for (auto& q : rest) srv->finish(std::move(q), TM_ECANCELED, "server stopped");
    (void)sync_stream(srv->st);
    (void)sync_stream(srv->bst);
    for (auto& kv : srv->cache) tm_weights_destroy(kv.second.w);
    srv->cache.clear();
    (void)sync_stream(srv->bst);
    (void)hipStreamDestroy(srv->st);
    (void)hipStreamDestroy(srv->bst);
    delete srv;
}
