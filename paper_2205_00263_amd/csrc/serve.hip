// Continuous-batching verification server behind query_submit / query_poll.
//
// One host thread runs the scheduler.  Every iteration it
//   1. admits waiting queries while problem slots and the memory budget allow
//      (their roots are bounded by bound_init, the DeepPoly pass);
//   2. for every problem (network x spec count x MNC use) gathers up to
//      max_batch pending subproblems, round-robin over live queries and lowest
//      lb first within a query, and bounds them with one bound_optimize call;
//   3. retires subproblems: ub < 0 on a spec row is a counterexample
//      (FALSIFIED), lb > 0 on every row verifies the subdomain; the others are
//      split on the neuron bound_optimize selects and their children join the
//      pending lists (Section 2.2 branch-and-bound, Section 3.2 splits);
//   4. finishes queries that are verified, falsified, out of time, out of
//      splittable neurons or over their subproblem cap.
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
    double timeout_s = 60.0;
};

struct Sub {
    int64_t id;
    float key;      // min over spec rows of lb
    int64_t order;  // creation order (ties)
};

struct Live {
    uint64_t ticket;
    int prob;                  // index into server problems
    QueryData data;
    std::vector<Sub> pending;  // waiting to be bounded
    int64_t in_flight = 0;     // in the current batch
    int64_t bounded = 0;
    float root_lb = -INFINITY;
    bool root_done = false;
    double t_submit = 0, t_admit = 0;
    int64_t created = 0;
};

struct ProbKey {
    int net, S, mnc;
    bool operator<(const ProbKey& o) const {
        return std::tie(net, S, mnc) < std::tie(o.net, o.S, o.mnc);
    }
};

}  // namespace

struct mnb_server {
    std::vector<mnb_net*> nets;
    mnb_server_cfg cfg;
    std::map<ProbKey, int> prob_of;
    std::vector<mnb_problem*> probs;
    std::vector<size_t> slot_bytes;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::pair<uint64_t, QueryData>> waiting;
    std::map<uint64_t, double> submit_time;
    std::map<uint64_t, mnb_result> finished;
    std::map<uint64_t, std::unique_ptr<Live>> live;   // worker-owned
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0 = Clock::now();
    std::string fatal;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    int problem_for(const QueryData& q);
    size_t used_bytes() const;
    void finish(Live& L, int verdict);
};

namespace {
constexpr int64_t kProblemCapacity = 8192;
}

int mnb_server::problem_for(const QueryData& q) {
    ProbKey k{q.net_index, q.n_spec, q.mnc.empty() ? 0 : 1};
    auto it = prob_of.find(k);
    if (it != prob_of.end()) return it->second;
    mnb_problem* pb = nullptr;
    int rc = mnb_problem_create(nets[q.net_index], q.n_spec, kProblemCapacity, k.mnc ? 500 : 0, &pb);
    if (rc != MNB_OK) throw mnb::Error{rc, std::string("server problem: ") + mnb_last_error()};
    probs.push_back(pb);
    const long sd = pb->ld_state, sp = pb->ld_param, sg = pb->ld_gamma;
    slot_bytes.push_back(sd * 9 + (size_t)pb->n_sets * (sp * 8 + sg * 4) + pb->S * 4 + 16);
    prob_of[k] = (int)probs.size() - 1;
    return (int)probs.size() - 1;
}

size_t mnb_server::used_bytes() const {
    size_t b = 0;
    for (size_t i = 0; i < probs.size(); ++i) b += (size_t)probs[i]->n_used * slot_bytes[i];
    return b;
}

void mnb_server::finish(Live& L, int verdict) {
    mnb_problem* pb = probs[L.prob];
    std::vector<int64_t> ids;
    for (auto& s : L.pending) ids.push_back(s.id);
    if (!ids.empty()) mnb_release(pb, ids.data(), (int)ids.size());
    L.pending.clear();
    mnb_result r{};
    r.verdict = verdict;
    r.lb = L.root_lb;
    r.subproblems = L.bounded;
    r.t_submit = L.t_submit;
    r.t_admit = L.t_admit;
    r.t_done = now();
    std::lock_guard<std::mutex> lk(mu);
    finished[L.ticket] = r;
}

void mnb_server::run() {
    for (;;) {
        // ---- admission
        std::vector<std::pair<uint64_t, QueryData>> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (waiting.empty() && live.empty()) cv.wait(lk, [&] { return stop || !waiting.empty(); });
            if (stop) return;
            while (!waiting.empty()) {
                admit.push_back(std::move(waiting.front()));
                waiting.pop_front();
            }
        }
        std::deque<std::pair<uint64_t, QueryData>> defer;
        for (auto& tq : admit) {
            QueryData& q = tq.second;
            int pi = problem_for(q);
            mnb_problem* pb = probs[pi];
            // memory: the root plus its first children must fit
            if (used_bytes() + 3 * slot_bytes[pi] > cfg.mem_budget || pb->free_list.size() < 3) {
                defer.push_back(std::move(tq));
                continue;
            }
            auto L = std::make_unique<Live>();
            L->ticket = tq.first;
            L->prob = pi;
            L->data = std::move(q);
            {
                std::lock_guard<std::mutex> lk(mu);
                L->t_submit = submit_time[L->ticket];
            }
            L->t_admit = now();
            std::vector<mnb_mnc> mv;
            for (auto& ml : L->data.mnc)
                mv.push_back(mnb_mnc{ml.layer, ml.e, ml.row_ptr.data(), ml.col.data(), ml.P.data(), ml.Phat.data(),
                                     ml.p.data()});
            std::vector<float> lb(L->data.n_spec), ub(L->data.n_spec);
            int64_t rid = -1;
            int rc = bound_init(pb, L->data.lo.data(), L->data.hi.data(), L->data.C.data(), L->data.c0.data(),
                                mv.empty() ? nullptr : mv.data(), (int)mv.size(), &rid, lb.data(), ub.data());
            L->bounded = 1;
            Live& R = *L;
            live[R.ticket] = std::move(L);
            if (rc != MNB_OK) {
                finish(R, MNB_UNKNOWN);
                live.erase(R.ticket);
                continue;
            }
            R.root_lb = *std::min_element(lb.begin(), lb.end());
            R.pending.push_back(Sub{rid, R.root_lb, R.created++});
            bool fals = false, ver = true;
            for (int s = 0; s < R.data.n_spec; ++s) {
                fals |= ub[s] < 0.f;
                ver &= lb[s] > 0.f;
            }
            if (fals || ver) {
                finish(R, fals ? MNB_FALSIFIED : MNB_VERIFIED);
                live.erase(R.ticket);
            }
        }
        if (!defer.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = defer.rbegin(); it != defer.rend(); ++it) waiting.push_front(std::move(*it));
        }
        if (live.empty()) {
            if (!defer.empty()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
            continue;
        }
        // ---- timeouts
        const double tnow = now();
        for (auto it = live.begin(); it != live.end();) {
            Live& L = *it->second;
            if (tnow - L.t_submit > L.data.timeout_s) {
                finish(L, MNB_TIMEOUT);
                it = live.erase(it);
            } else {
                ++it;
            }
        }
        // ---- one batch per problem
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
            int rc = bound_optimize(pb, ids.data(), n, &cfg.opt, lb.data(), ub.data(), bl.data(), bn.data());
            if (rc != MNB_OK) {
                for (auto& o : owner) {
                    Live* L = o.first;
                    if (live.count(L->ticket)) {
                        mnb_release(pb, &o.second.id, 1);
                        finish(*L, MNB_UNKNOWN);
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
            std::vector<int64_t> par, rel;
            std::vector<int32_t> lay, neu;
            std::vector<Live*> par_owner;
            std::map<Live*, int> verdict;
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
                    verdict[L] = MNB_FALSIFIED;
                    rel.push_back(ids[b]);
                } else if (ver) {
                    rel.push_back(ids[b]);
                } else if (bl[b] < 0) {
                    verdict[L] = MNB_UNKNOWN;
                    rel.push_back(ids[b]);
                } else {
                    par.push_back(ids[b]);
                    lay.push_back(bl[b]);
                    neu.push_back(bn[b]);
                    par_owner.push_back(L);
                }
            }
            // drop splits of queries that just finished
            std::vector<int64_t> par2;
            std::vector<int32_t> lay2, neu2;
            std::vector<Live*> own2;
            for (size_t k = 0; k < par.size(); ++k) {
                if (verdict.count(par_owner[k])) {
                    rel.push_back(par[k]);
                    continue;
                }
                Live* L = par_owner[k];
                if ((int64_t)L->pending.size() + 2 > cfg.queue_cap || pb->free_list.size() < 2 * (par2.size() + 1) ||
                    used_bytes() + 2 * (par2.size() + 1) * slot_bytes[pi] > cfg.mem_budget) {
                    verdict[L] = MNB_UNKNOWN;
                    rel.push_back(par[k]);
                    continue;
                }
                par2.push_back(par[k]);
                lay2.push_back(lay[k]);
                neu2.push_back(neu[k]);
                own2.push_back(L);
            }
            if (!par2.empty()) {
                std::vector<int64_t> kids(2 * par2.size());
                rc = branch_split(pb, par2.data(), lay2.data(), neu2.data(), (int)par2.size(), kids.data());
                if (rc == MNB_OK) {
                    for (size_t k = 0; k < par2.size(); ++k) {
                        Live* L = own2[k];
                        if (verdict.count(L)) {
                            rel.push_back(kids[2 * k]);
                            rel.push_back(kids[2 * k + 1]);
                            continue;
                        }
                        float key = INFINITY;
                        for (size_t b = 0; b < ids.size(); ++b)
                            if (ids[b] == par2[k])
                                for (int s = 0; s < S; ++s) key = std::min(key, lb[b * S + s]);
                        L->pending.push_back(Sub{kids[2 * k], key, L->created++});
                        L->pending.push_back(Sub{kids[2 * k + 1], key, L->created++});
                    }
                } else {
                    for (Live* L : own2) verdict[L] = MNB_UNKNOWN;
                }
                rel.insert(rel.end(), par2.begin(), par2.end());
            }
            if (!rel.empty()) mnb_release(pb, rel.data(), (int)rel.size());
            for (auto& kv : verdict) {
                finish(*kv.first, kv.second);
                live.erase(kv.first->ticket);
            }
            // queries with nothing left pending and nothing refuted are verified
            for (auto it = live.begin(); it != live.end();) {
                Live& L = *it->second;
                if (L.prob == (int)pi && L.pending.empty()) {
                    finish(L, MNB_VERIFIED);
                    it = live.erase(it);
                } else {
                    ++it;
                }
            }
        }
    }
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
        std::lock_guard<std::mutex> lk(s->mu);
        MNB_CHECK(s->fatal.empty(), MNB_ESTATE, "server stopped: " + s->fatal);
        *ticket = s->next_ticket++;
        s->submit_time[*ticket] = s->now();
        s->waiting.emplace_back(*ticket, std::move(d));
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
