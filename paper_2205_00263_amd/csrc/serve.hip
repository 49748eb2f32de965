// Continuous-batching verification server behind query_submit / query_poll.
//
// One host thread runs the scheduler.  Every iteration it
//   1. splits parked parents (bounded subproblems that found no room for their
//      children), oldest query first, as far as slots and memory allow;
//   2. admits waiting queries while slots and the memory budget allow beyond
//      what parked splits need (their roots are bounded by bound_init, the
//      DeepPoly pass; constraints are generated on the device when asked);
//   3. for every problem (network x spec count x constraint use) gathers up to
//      max_batch pending subproblems, round-robin over live queries and lowest
//      lb first within a query, and bounds them with one bound_optimize call;
//   4. retires subproblems: ub < 0 on a spec row is a counterexample
//      (FALSIFIED), lb > 0 on every row verifies the subdomain; the others are
//      split on the neuron bound_optimize selects (Section 2.2 branch-and-bound,
//      Section 3.2 splits) or parked when there is no room;
//   5. finishes queries that are verified, falsified, out of time, out of
//      splittable neurons or over their subproblem cap; if nothing could be
//      bounded or split, preempts the most recently admitted query holding slots
//      (it starts over later), or ends a query alone on the server as out of
//      memory.
// Queries that arrive while a batch runs join at the next iteration, so their
// work shares the device with the subproblems already in flight.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "engine.h"

namespace {

using Clock = std::chrono::steady_clock;

struct QueryData {
    int net_index = 0, n_spec = 0;
    std::vector<float> lo, hi, C, c0;
    struct Layer {
        int layer, e;
        std::vector<int32_t> row_ptr, col;
        std::vector<float> P, Phat, p;
    };
    std::vector<Layer> mnc;
    int mnc_cap = 0;
    double timeout_s = 60.0;
};

struct Sub {
    int64_t id;
    float key;      // min over spec rows of lb
    int64_t order;  // creation order (ties)
};
struct Parked {
    Sub sub;
    int32_t layer, neuron;   // the split bound_optimize chose
};

struct Waiting {
    uint64_t ticket;
    QueryData data;
    int restarts = 0;
};

struct Live {
    uint64_t ticket;
    int prob;                  // index into server problems
    QueryData data;
    std::vector<Sub> pending;  // waiting to be bounded
    std::vector<Parked> parked;
    int64_t bounded = 0;
    float root_lb = -INFINITY;
    bool root_done = false;
    double t_submit = 0, t_admit = 0;
    int64_t created = 0;
    uint64_t admit_seq = 0;
    int restarts = 0;
    int64_t held() const { return (int64_t)pending.size() + (int64_t)parked.size(); }
};

struct ProbKey {
    int net, S, mnc;
    bool operator<(const ProbKey& o) const { return std::tie(net, S, mnc) < std::tie(o.net, o.S, o.mnc); }
};

constexpr int64_t kInitialSlots = 256;   // a pool starts with at most this many slots and doubles on demand
constexpr int64_t kMaxSlots = 1 << 20;
constexpr int kServerMaxMnc = 500;

// Device bytes of one subproblem slot of a problem on `net` (mnb::problem_slot_bytes before it exists).
size_t slot_bytes_for(const mnb_net* net, int n_spec, bool with_mnc) {
    const long ld = (net->total_d + 15) / 16 * 16, n_sets = 2 * (long)net->relus.size() - 1;
    const long ldg = ((long)net->relus.size() * (with_mnc ? kServerMaxMnc : 0) + 15) / 16 * 16;
    return (size_t)ld * 9 + (size_t)n_sets * (ld * 8 + ldg * 4) + 4 + (size_t)n_spec * 4;
}

}  // namespace

struct mnb_server {
    std::vector<mnb_net*> nets;
    mnb_server_cfg cfg;
    std::map<ProbKey, int> prob_of;
    std::vector<mnb_problem*> probs;
    std::vector<size_t> slot_bytes;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Waiting> waiting;
    std::map<uint64_t, double> submit_time;
    std::map<uint64_t, mnb_result> finished;
    std::map<uint64_t, std::unique_ptr<Live>> live;   // worker-owned
    uint64_t next_ticket = 1, admit_counter = 0;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0 = Clock::now();
    std::string fatal, last_error;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    bool iterate();
    int problem_for(const QueryData& q);
    size_t committed_bytes() const;
    bool ensure_free(int pi, int64_t need);
    void finish_ticket(uint64_t ticket, int verdict, int reason, float lb, int64_t bounded, double t_submit,
                       double t_admit, int restarts);
    void finish(Live& L, int verdict, int reason);
    void preempt(Live& L);
    bool admit(Waiting& w);
};

// Device bytes the server holds: every slot pool and every problem's workspace.
size_t mnb_server::committed_bytes() const {
    size_t b = 0;
    for (size_t i = 0; i < probs.size(); ++i) b += (size_t)probs[i]->cap * slot_bytes[i] + probs[i]->ws.total();
    return b;
}

int mnb_server::problem_for(const QueryData& q) {
    const bool with_mnc = !q.mnc.empty() || q.mnc_cap > 0;
    ProbKey k{q.net_index, q.n_spec, with_mnc ? 1 : 0};
    auto it = prob_of.find(k);
    if (it != prob_of.end()) return it->second;
    // the first pool takes at most a quarter of the budget; it grows on demand
    const size_t sb = slot_bytes_for(nets[q.net_index], q.n_spec, with_mnc);
    int64_t cap0 = std::max<int64_t>(3, std::min<int64_t>(kInitialSlots, (int64_t)(cfg.mem_budget / 4 / sb)));
    if (cfg.max_slots > 0) cap0 = std::min(cap0, std::max<int64_t>(3, cfg.max_slots));
    if (committed_bytes() + (size_t)cap0 * sb > cfg.mem_budget)
        throw mnb::Error{MNB_ENOMEM, "server: no room for another slot pool within mem_budget"};
    mnb_problem* pb = nullptr;
    int rc = mnb_problem_create(nets[q.net_index], q.n_spec, cap0, with_mnc ? kServerMaxMnc : 0, &pb);
    if (rc != MNB_OK) throw mnb::Error{rc, std::string("server problem: ") + mnb_last_error()};
    probs.push_back(pb);
    slot_bytes.push_back(mnb::problem_slot_bytes(pb));
    prob_of[k] = (int)probs.size() - 1;
    return (int)probs.size() - 1;
}

// At least `need` free slots in problem pi, doubling its pool while the budget allows.
bool mnb_server::ensure_free(int pi, int64_t need) {
    mnb_problem* pb = probs[pi];
    while ((int64_t)pb->free_list.size() < need) {
        const int64_t lim = cfg.max_slots > 0 ? std::min<int64_t>(kMaxSlots, cfg.max_slots) : kMaxSlots;
        const int64_t nc = std::min<int64_t>(lim, std::max<int64_t>(2 * pb->cap, pb->cap + need));
        if (nc <= pb->cap) return false;
        if (committed_bytes() + (size_t)(nc - pb->cap) * slot_bytes[pi] > cfg.mem_budget) return false;
        try {
            mnb::problem_grow(pb, nc);
        } catch (const mnb::Error& e) {
            last_error = e.msg;
            return false;
        }
    }
    return true;
}

void mnb_server::finish_ticket(uint64_t ticket, int verdict, int reason, float lb, int64_t bounded, double t_submit,
                               double t_admit, int restarts) {
    mnb_result r{};
    r.verdict = verdict;
    r.reason = reason;
    r.lb = lb;
    r.subproblems = bounded;
    r.t_submit = t_submit;
    r.t_admit = t_admit;
    r.t_done = now();
    r.restarts = restarts;
    std::lock_guard<std::mutex> lk(mu);
    finished[ticket] = r;
}

void mnb_server::finish(Live& L, int verdict, int reason) {
    mnb_problem* pb = probs[L.prob];
    std::vector<int64_t> ids;
    for (auto& s : L.pending) ids.push_back(s.id);
    for (auto& p : L.parked) ids.push_back(p.sub.id);
    if (!ids.empty()) mnb_release(pb, ids.data(), (int)ids.size());
    L.pending.clear();
    L.parked.clear();
    finish_ticket(L.ticket, verdict, reason, L.root_lb, L.bounded, L.t_submit, L.t_admit, L.restarts);
}

// Release a live query's subproblems and queue it again at the front; it starts over when admitted.
void mnb_server::preempt(Live& L) {
    mnb_problem* pb = probs[L.prob];
    std::vector<int64_t> ids;
    for (auto& s : L.pending) ids.push_back(s.id);
    for (auto& p : L.parked) ids.push_back(p.sub.id);
    if (!ids.empty()) mnb_release(pb, ids.data(), (int)ids.size());
    Waiting w;
    w.ticket = L.ticket;
    w.data = std::move(L.data);
    w.restarts = L.restarts + 1;
    std::lock_guard<std::mutex> lk(mu);
    waiting.push_front(std::move(w));
}

// Admit one waiting query: false if it has to keep waiting (no room yet).
bool mnb_server::admit(Waiting& w) {
    QueryData& q = w.data;
    double t_submit;
    {
        std::lock_guard<std::mutex> lk(mu);
        t_submit = submit_time[w.ticket];
    }
    int pi;
    try {
        pi = problem_for(q);
    } catch (const mnb::Error& e) {
        last_error = e.msg;
        finish_ticket(w.ticket, MNB_UNKNOWN, MNB_R_ERROR, -INFINITY, 0, t_submit, now(), w.restarts);
        return true;
    }
    mnb_problem* pb = probs[pi];
    // room for the root and its first children beyond what the parked splits of this problem need
    int64_t parked = 0;
    for (auto& kv : live)
        if (kv.second->prob == pi) parked += 2 * (int64_t)kv.second->parked.size();
    if (!ensure_free(pi, parked + 3)) return false;
    auto L = std::make_unique<Live>();
    L->ticket = w.ticket;
    L->prob = pi;
    L->data = std::move(q);
    L->t_submit = t_submit;
    L->t_admit = now();
    L->admit_seq = ++admit_counter;
    L->restarts = w.restarts;
    std::vector<mnb_mnc> mv;
    for (auto& ml : L->data.mnc)
        mv.push_back(mnb_mnc{ml.layer, ml.e, ml.row_ptr.data(), ml.col.data(), ml.P.data(), ml.Phat.data(), ml.p.data()});
    std::vector<float> lb(L->data.n_spec), ub(L->data.n_spec);
    int64_t rid = -1;
    int rc = bound_init(pb, L->data.lo.data(), L->data.hi.data(), L->data.C.data(), L->data.c0.data(),
                        mv.empty() ? nullptr : mv.data(), (int)mv.size(), &rid, lb.data(), ub.data());
    L->bounded = 1;
    Live& R = *L;
    live[R.ticket] = std::move(L);
    if (rc == MNB_OK && R.data.mnc.empty() && R.data.mnc_cap > 0) {
        rc = mnb_mnc_generate(pb, rid, std::min(R.data.mnc_cap, kServerMaxMnc), nullptr);
        if (rc != MNB_OK) mnb_release(pb, &rid, 1);
    }
    if (rc != MNB_OK) {
        last_error = mnb_last_error();
        finish(R, MNB_UNKNOWN, MNB_R_ERROR);
        live.erase(R.ticket);
        return true;
    }
    R.root_lb = *std::min_element(lb.begin(), lb.end());
    R.pending.push_back(Sub{rid, R.root_lb, R.created++});
    bool fals = false, ver = true;
    for (int s = 0; s < R.data.n_spec; ++s) {
        fals |= ub[s] < 0.f;
        ver &= lb[s] > 0.f;
    }
    if (fals || ver) {
        finish(R, fals ? MNB_FALSIFIED : MNB_VERIFIED, MNB_R_NONE);
        live.erase(R.ticket);
    }
    return true;
}

void mnb_server::run() {
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (waiting.empty() && live.empty()) cv.wait(lk, [&] { return stop || !waiting.empty(); });
            if (stop) return;
        }
        if (!iterate()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
}

// One scheduler iteration; returns whether anything was bounded, split or finished.
bool mnb_server::iterate() {
    bool progress = false;
    // ---- parked splits first (oldest query first)
    {
        std::vector<Live*> order;
        for (auto& kv : live)
            if (!kv.second->parked.empty()) order.push_back(kv.second.get());
        std::sort(order.begin(), order.end(), [](Live* a, Live* b) { return a->admit_seq < b->admit_seq; });
        for (Live* L : order) {
            mnb_problem* pb = probs[L->prob];
            size_t k = 0;
            for (; k < L->parked.size(); ++k) {
                if (!ensure_free(L->prob, 2)) break;
                const Parked& P = L->parked[k];
                int64_t kids[2];
                if (branch_split(pb, &P.sub.id, &P.layer, &P.neuron, 1, kids) != MNB_OK) break;
                mnb_release(pb, &P.sub.id, 1);
                L->pending.push_back(Sub{kids[0], P.sub.key, L->created++});
                L->pending.push_back(Sub{kids[1], P.sub.key, L->created++});
                progress = true;
            }
            L->parked.erase(L->parked.begin(), L->parked.begin() + k);
        }
    }
    // ---- admission and timeouts of waiting queries
    {
        std::deque<Waiting> todo;
        {
            std::lock_guard<std::mutex> lk(mu);
            todo.swap(waiting);
        }
        std::deque<Waiting> defer;
        const double tnow = now();
        while (!todo.empty()) {
            Waiting w = std::move(todo.front());
            todo.pop_front();
            double t_submit;
            {
                std::lock_guard<std::mutex> lk(mu);
                t_submit = submit_time[w.ticket];
            }
            if (tnow - t_submit > w.data.timeout_s) {
                finish_ticket(w.ticket, MNB_TIMEOUT, MNB_R_TIME, -INFINITY, 0, t_submit, tnow, w.restarts);
                progress = true;
                continue;
            }
            if (!defer.empty() || !admit(w)) {   // first come, first served
                defer.push_back(std::move(w));
                continue;
            }
            progress = true;
        }
        if (!defer.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = defer.rbegin(); it != defer.rend(); ++it) waiting.push_front(std::move(*it));
        }
    }
    if (live.empty()) return progress;
    // ---- timeouts
    const double tnow = now();
    for (auto it = live.begin(); it != live.end();) {
        Live& L = *it->second;
        if (tnow - L.t_submit > L.data.timeout_s) {
            finish(L, MNB_TIMEOUT, MNB_R_TIME);
            it = live.erase(it);
            progress = true;
        } else {
            ++it;
        }
    }
    // ---- one batch per problem
    mnb_opt_cfg opt = cfg.opt;
    if (opt.mem_budget == 0) opt.mem_budget = cfg.mem_budget / 4;
    for (size_t pi = 0; pi < probs.size(); ++pi) {
        std::vector<Live*> qs;
        for (auto& kv : live)
            if (kv.second->prob == (int)pi && !kv.second->pending.empty()) qs.push_back(kv.second.get());
        if (qs.empty()) continue;
        for (Live* L : qs)
            std::sort(L->pending.begin(), L->pending.end(), [](const Sub& a, const Sub& b) {
                return a.key < b.key || (a.key == b.key && a.order < b.order);
            });
        std::vector<int64_t> ids;
        std::vector<std::pair<Live*, Sub>> owner;
        std::vector<size_t> cursor(qs.size(), 0);
        bool more = true;
        while ((int)ids.size() < cfg.max_batch && more) {
            more = false;
            for (size_t k = 0; k < qs.size() && (int)ids.size() < cfg.max_batch; ++k) {
                if (cursor[k] < qs[k]->pending.size()) {
                    const Sub& s = qs[k]->pending[cursor[k]++];
                    ids.push_back(s.id);
                    owner.push_back({qs[k], s});
                    more = true;
                }
            }
        }
        for (size_t k = 0; k < qs.size(); ++k)
            qs[k]->pending.erase(qs[k]->pending.begin(), qs[k]->pending.begin() + cursor[k]);
        mnb_problem* pb = probs[pi];
        const int S = pb->S, n = (int)ids.size();
        std::vector<float> lb((size_t)n * S), ub((size_t)n * S);
        std::vector<int32_t> bl(n), bn(n);
        int rc = bound_optimize(pb, ids.data(), n, &opt, lb.data(), ub.data(), bl.data(), bn.data());
        progress = true;
        if (rc != MNB_OK) {
            last_error = mnb_last_error();
            for (auto& o : owner) {
                Live* L = o.first;
                mnb_release(pb, &o.second.id, 1);
                if (live.count(L->ticket)) {
                    finish(*L, MNB_UNKNOWN, MNB_R_ERROR);
                    live.erase(L->ticket);
                }
            }
            continue;
        }
        if (pb->has_mnc) {
            // with multi-neuron constraints: cost adjusted active constraint branching
            // (Section 3.4); a subproblem whose constraints carry no weight (score 0, e.g. a
            // query without constraints) keeps the alpha-contribution choice
            std::vector<int32_t> al(n), an(n);
            std::vector<float> as(n);
            if (mnb::branch_acs_cab(pb, ids.data(), n, al.data(), an.data(), as.data()) == MNB_OK)
                for (int b = 0; b < n; ++b)
                    if (al[b] >= 0 && as[b] > 0.f) {
                        bl[b] = al[b];
                        bn[b] = an[b];
                    }
        }
        std::vector<int64_t> rel;
        std::map<Live*, std::pair<int, int>> verdict;   // verdict, reason
        std::vector<std::pair<Live*, Parked>> want;    // subproblems to split
        for (int b = 0; b < n; ++b) {
            Live* L = owner[b].first;
            L->bounded++;
            if (verdict.count(L)) {
                rel.push_back(ids[b]);
                continue;
            }
            bool fals = false, ver = true;
            float key = INFINITY;
            for (int s = 0; s < S; ++s) {
                fals |= ub[(size_t)b * S + s] < 0.f;
                ver &= lb[(size_t)b * S + s] > 0.f;
                key = std::min(key, lb[(size_t)b * S + s]);
            }
            if (!L->root_done && owner[b].second.order == 0) {
                L->root_lb = key;
                L->root_done = true;
            }
            if (fals) {
                verdict[L] = {MNB_FALSIFIED, MNB_R_NONE};
                rel.push_back(ids[b]);
            } else if (ver) {
                rel.push_back(ids[b]);
            } else if (bl[b] < 0) {
                verdict[L] = {MNB_UNKNOWN, MNB_R_NO_SPLIT};
                rel.push_back(ids[b]);
            } else {
                want.push_back({L, Parked{Sub{ids[b], key, owner[b].second.order}, bl[b], bn[b]}});
            }
        }
        // split where there is room; park the rest (their queries' own caps still apply)
        std::vector<int64_t> par;
        std::vector<int32_t> lay, neu;
        std::vector<std::pair<Live*, float>> par_owner;
        for (auto& w : want) {
            Live* L = w.first;
            if (verdict.count(L)) {
                rel.push_back(w.second.sub.id);
                continue;
            }
            if (L->held() + 2 > cfg.queue_cap) {
                verdict[L] = {MNB_UNKNOWN, MNB_R_QUEUE_CAP};
                rel.push_back(w.second.sub.id);
                continue;
            }
            if (!L->parked.empty() || !ensure_free((int)pi, 2 * (int64_t)(par.size() + 1))) {
                L->parked.push_back(w.second);
                continue;
            }
            par.push_back(w.second.sub.id);
            lay.push_back(w.second.layer);
            neu.push_back(w.second.neuron);
            par_owner.push_back({L, w.second.sub.key});
        }
        if (!par.empty()) {
            std::vector<int64_t> kids(2 * par.size());
            rc = branch_split(pb, par.data(), lay.data(), neu.data(), (int)par.size(), kids.data());
            if (rc == MNB_OK) {
                for (size_t k = 0; k < par.size(); ++k) {
                    Live* L = par_owner[k].first;
                    if (verdict.count(L)) {
                        rel.push_back(kids[2 * k]);
                        rel.push_back(kids[2 * k + 1]);
                        continue;
                    }
                    L->pending.push_back(Sub{kids[2 * k], par_owner[k].second, L->created++});
                    L->pending.push_back(Sub{kids[2 * k + 1], par_owner[k].second, L->created++});
                }
            } else {
                last_error = mnb_last_error();
                for (auto& po : par_owner) verdict[po.first] = {MNB_UNKNOWN, MNB_R_ERROR};
            }
            rel.insert(rel.end(), par.begin(), par.end());
        }
        if (!rel.empty()) mnb_release(pb, rel.data(), (int)rel.size());
        for (auto& kv : verdict) {
            finish(*kv.first, kv.second.first, kv.second.second);
            live.erase(kv.first->ticket);
        }
        // queries with nothing left pending or parked and nothing refuted are verified
        for (auto it = live.begin(); it != live.end();) {
            Live& L = *it->second;
            if (L.prob == (int)pi && L.pending.empty() && L.parked.empty()) {
                finish(L, MNB_VERIFIED, MNB_R_NONE);
                it = live.erase(it);
            } else {
                ++it;
            }
        }
    }
    if (!progress && !live.empty()) {
        // nothing could be bounded or split: every live subproblem waits for room.  Preempt the most
        // recently admitted query holding slots; alone on the server, a query is out of memory.
        Live* young = nullptr;
        for (auto& kv : live)
            if (kv.second->held() > 0 && (!young || kv.second->admit_seq > young->admit_seq)) young = kv.second.get();
        if (young) {
            if (live.size() == 1) {
                finish(*young, MNB_UNKNOWN, MNB_R_MEMORY);
            } else {
                preempt(*young);
            }
            live.erase(young->ticket);
            progress = true;
        }
    }
    return progress;
}

// =====================================================================================
// C ABI
// =====================================================================================
extern "C" void mnb_server_cfg_default(mnb_server_cfg* c) {
    if (!c) return;
    mnb_opt_cfg_default(&c->opt);
    c->max_batch = 256;
    c->queue_cap = 4096;
    c->mem_budget = (size_t)64 << 30;
    c->max_slots = 0;
}

extern "C" int mnb_server_create(mnb_net* const* nets, int n_nets, const mnb_server_cfg* cfg, mnb_server** out) {
    try {
        MNB_CHECK(nets && n_nets > 0 && out, MNB_EINVAL, "bad arguments");
        for (int i = 0; i < n_nets; ++i) MNB_CHECK(nets[i], MNB_EINVAL, "null net");
        auto s = new mnb_server();
        s->nets.assign(nets, nets + n_nets);
        if (cfg)
            s->cfg = *cfg;
        else
            mnb_server_cfg_default(&s->cfg);
        if (s->cfg.max_batch <= 0) s->cfg.max_batch = 256;
        if (s->cfg.queue_cap <= 0) s->cfg.queue_cap = 4096;
        if (s->cfg.mem_budget == 0) s->cfg.mem_budget = (size_t)64 << 30;
        s->worker = std::thread([s] {
            try {
                s->run();
            } catch (const mnb::Error& e) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->fatal = e.msg;
            } catch (const std::exception& e) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->fatal = e.what();
            }
        });
        *out = s;
    } catch (const mnb::Error& e) {
        mnb::set_error(e.code, e.msg);
        return e.code;
    }
    return MNB_OK;
}

extern "C" void mnb_server_destroy(mnb_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto* pb : s->probs) mnb_problem_destroy(pb);
    delete s;
}

extern "C" int query_submit(mnb_server* s, const mnb_query* q, uint64_t* ticket) {
    try {
        MNB_CHECK(s && q && ticket, MNB_EINVAL, "null argument");
        MNB_CHECK(q->net_index >= 0 && q->net_index < (int)s->nets.size(), MNB_EINVAL, "bad net_index");
        MNB_CHECK(q->n_spec > 0 && q->x_lo && q->x_hi && q->C && q->c0, MNB_EINVAL, "bad query arrays");
        const mnb_net* net = s->nets[q->net_index];
        QueryData d;
        d.net_index = q->net_index;
        d.n_spec = q->n_spec;
        d.lo.assign(q->x_lo, q->x_lo + net->d0);
        d.hi.assign(q->x_hi, q->x_hi + net->d0);
        d.C.assign(q->C, q->C + (size_t)q->n_spec * net->n_out);
        d.c0.assign(q->c0, q->c0 + q->n_spec);
        d.timeout_s = q->timeout_s > 0 ? q->timeout_s : 60.0;
        MNB_CHECK(q->mnc_cap >= 0 && q->mnc_cap <= 500, MNB_EINVAL, "server: mnc_cap must be in [0, 500]");
        d.mnc_cap = q->n_mnc > 0 ? 0 : q->mnc_cap;
        for (int i = 0; i < q->n_mnc; ++i) {
            const mnb_mnc& m = q->mnc[i];
            QueryData::Layer L;
            L.layer = m.layer;
            L.e = m.e;
            MNB_CHECK(m.e >= 0 && m.e <= 500, MNB_EINVAL, "server: at most 500 MNC rows per layer");
            if (m.e > 0) {
                const int nnz = m.row_ptr[m.e];
                L.row_ptr.assign(m.row_ptr, m.row_ptr + m.e + 1);
                L.col.assign(m.col, m.col + nnz);
                L.P.assign(m.P, m.P + nnz);
                L.Phat.assign(m.Phat, m.Phat + nnz);
                L.p.assign(m.p, m.p + m.e);
            }
            d.mnc.push_back(std::move(L));
        }
        MNB_CHECK(3 * slot_bytes_for(net, q->n_spec, !d.mnc.empty() || d.mnc_cap > 0) <= s->cfg.mem_budget,
                  MNB_EINVAL, "server: a root and two children of this query need more than mem_budget");
        std::lock_guard<std::mutex> lk(s->mu);
        MNB_CHECK(s->fatal.empty(), MNB_ESTATE, "server stopped: " + s->fatal);
        *ticket = s->next_ticket++;
        s->submit_time[*ticket] = s->now();
        Waiting w;
        w.ticket = *ticket;
        w.data = std::move(d);
        s->waiting.push_back(std::move(w));
    } catch (const mnb::Error& e) {
        mnb::set_error(e.code, e.msg);
        return e.code;
    }
    s->cv.notify_all();
    return MNB_OK;
}

extern "C" int query_poll(mnb_server* s, uint64_t ticket, mnb_result* out) {
    if (!s || !out) {
        mnb::set_error(MNB_EINVAL, "null argument");
        return MNB_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->finished.find(ticket);
    if (it != s->finished.end()) {
        *out = it->second;
        return MNB_OK;
    }
    if (!s->fatal.empty()) {
        mnb::set_error(MNB_ESTATE, "server stopped: " + s->fatal);
        return MNB_ESTATE;
    }
    if (ticket == 0 || ticket >= s->next_ticket) {
        mnb::set_error(MNB_EINVAL, "unknown ticket");
        return MNB_EINVAL;
    }
    return MNB_PENDING;
}
