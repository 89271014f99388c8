// Serving (include/qnae.h, qnae_server_*): continuous batching of QAOA solve
// requests on one GPU, driven by a host scheduler thread.
//
// Memory: one device pool split by a buddy allocator (every state is a power
// of two of 8-byte amplitudes, so blocks do not fragment into odd sizes).
// Each active request holds a cost block; a large one (n > 14) also holds a
// state block and an aux block (phase tables, mixer forms, tile partial sums).
// Requests are NAE instances, so a large one is solved on the half state
// (x < 2^(n-1), the global-flip symmetry): half the pool and the traffic.
//
// Tick: admit queued requests (FIFO) while a slot is free and the pool can
// hold them; upload everything new in one pinned copy; build the new cost
// diagonals (one batched launch); run new small requests whole (one batched
// resident launch); advance the large requests by one or more rounds of one
// sweep each (one batched launch per round, sweep kind and cost type); read
// out requests whose plan ended (one batched reduce), copy all results back
// in one copy, free their blocks and wake their waiters.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "host.h"

using namespace qnae_host;
using qnae::ClauseRec;
using qnae::MixForm;
using qnae::SweepArgs;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Buddy allocator over [0, 2^max_order) in blocks of 2^order bytes.
class Buddy {
   public:
    static constexpr int kMinOrder = 12;
    explicit Buddy(int max_order) : max_order_(max_order), free_(max_order + 1) { free_[max_order].insert(0); }
    static int order_for(uint64_t bytes) {
        int o = kMinOrder;
        while ((1ull << o) < bytes) ++o;
        return o;
    }
    bool alloc(int order, uint64_t* off) {
        int o = order;
        while (o <= max_order_ && free_[o].empty()) ++o;
        if (o > max_order_) return false;
        uint64_t at = *free_[o].begin();
        free_[o].erase(free_[o].begin());
        while (o > order) {  // split, keep the lower half
            --o;
            free_[o].insert(at + (1ull << o));
        }
        used_ += 1ull << order;
        peak_ = std::max(peak_, used_);
        *off = at;
        return true;
    }
    void release(uint64_t at, int order) {
        used_ -= 1ull << order;
        while (order < max_order_) {
            const uint64_t buddy = at ^ (1ull << order);
            auto it = free_[order].find(buddy);
            if (it == free_[order].end()) break;
            free_[order].erase(it);
            at = std::min(at, buddy);
            ++order;
        }
        free_[order].insert(at);
    }
    uint64_t peak() const { return peak_; }
    uint64_t used() const { return used_; }

   private:
    int max_order_;
    std::vector<std::set<uint64_t>> free_;
    uint64_t used_ = 0, peak_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    int n = 0, m = 0, k = 0, p = 0, dtype = QNAE_U8;
    std::vector<int32_t> clauses;
    std::vector<double> gammas, betas;
    double t_submit = 0, t_done = 0;
    enum { QUEUED, ACTIVE, DONE, FAILED, CANCELED } state = QUEUED;
    bool cancel = false;  // drop before the next tick
    qnae_result result{};
    // active
    bool resident = false;
    bool half = false;  // state and cost kept for x < 2^(n-1) (NAE global-flip symmetry)
    uint64_t state_off = 0, cost_off = 0, aux_off = 0;
    int state_order = -1, cost_order = -1, aux_order = -1;
    size_t form_off = 0, part_off = 0;  // inside the aux block (tables at 0)
    uint32_t tiles = 0;
    qnae_tune shape{};  // tile shape of its sweeps (the context's tuned shape for its n)
    SweepPlan plan;
    std::complex<double> final_scale;
    size_t next_op = 0;
    bool cost_built = false;
};

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct qnae_server {
    qnae_ctx* ctx = nullptr;
    int device = 0;
    // the context's tile shapes when the server was made: tuned shapes per
    // (n, cost type) and the default (read on the scheduler thread, so a copy)
    std::map<std::pair<int, int>, qnae_tune> tunes;
    qnae_tune default_shape{};
    int max_slots = 1;
    hipStream_t stream = nullptr;
    char* pool = nullptr;
    uint64_t pool_bytes = 0;
    std::unique_ptr<Buddy> buddy;
    DevBuf d_blob;
    HostBuf h_blob;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    int error = QNAE_OK;
    std::string error_msg;
    uint64_t completed = 0, ticks = 0, launches = 0;
    double tick_bytes = 8e9;  // state traffic per tick, about 1.5 ms of HBM time
    bool use_half = true;     // half-state solves for requests with n > 14 (QNAE_SERVER_HALF)
    // QNAE_FAULT_INJECT=server_tick:K makes tick K (1-based) fail as a device
    // error would, before it launches anything: for tests of failure handling.
    uint64_t fault_tick = 0;
    std::thread worker;

    // Footprint blocks of a request (-1: none); false if it can never fit.
    // Large requests: state, cost, aux = [tables | forms | tile partials].
    // Small (resident) requests: cost only; their tables stay in the upload.
    bool plan_blocks(Request& r, int* so, int* co, int* ao) const {
        const uint64_t N = 1ull << (r.n - (r.half ? 1 : 0));
        const int T = r.p > 0 ? r.p : 1;
        r.form_off = round_up(sizeof(float2) * (uint64_t)T * (r.m + 1), 256);
        r.part_off = r.form_off + round_up(sizeof(MixForm) * T, 256);
        *co = Buddy::order_for(N * (r.dtype == QNAE_U8 ? 1 : 2));
        *so = r.resident ? -1 : Buddy::order_for(N * 8);
        *ao = r.resident ? -1 : Buddy::order_for(r.part_off + sizeof(double) * 3 * (uint64_t)r.tiles);
        const uint64_t total = (1ull << *co) + (*ao >= 0 ? 1ull << *ao : 0) + (*so >= 0 ? 1ull << *so : 0);
        return total <= pool_bytes;
    }
    void release(Request& r) {
        if (r.state_order >= 0) buddy->release(r.state_off, r.state_order);
        if (r.cost_order >= 0) buddy->release(r.cost_off, r.cost_order);
        if (r.aux_order >= 0) buddy->release(r.aux_off, r.aux_order);
        r.state_order = r.cost_order = r.aux_order = -1;
    }
    int tick(std::vector<Request*>& admitted);
    void run();
};

namespace {

int fail_server(qnae_server* S, int code) {
    std::lock_guard<std::mutex> g(S->mu);
    S->error = code;
    S->error_msg = last_error();
    return code;
}

}  // namespace

// One scheduler tick over the requests admitted now and the active ones. A
// tick runs several rounds (each round advances every unfinished large
// request by one sweep) while the rounds' state traffic stays within
// tick_bytes, so that a lightly loaded server does not pay one host
// round trip per sweep, and a heavily loaded one still admits new requests
// often.
int qnae_server::tick(std::vector<Request*>& admitted) try {
    hipStream_t s = stream;
    if (fault_tick && ticks + 1 == fault_tick) return fail(QNAE_EHIP, "injected fault at scheduler tick %llu",
                                                           (unsigned long long)fault_tick);
    Blob B;
    // Host side of new requests: clause records, tables, plans. Tables go
    // through the upload blob; large requests copy them on into their aux
    // block, small ones read them there.
    struct New {
        Request* r;
        size_t rec_at, tab_at;
        int nrec, nlow = 0;
        std::vector<ClauseRec> recs;
        std::vector<float2> tabs;
        std::vector<MixForm> forms;
    };
    std::vector<New> nw(admitted.size());
    for (size_t i = 0; i < admitted.size(); ++i) {
        Request& r = *admitted[i];
        New& w = nw[i];
        w.r = &r;
        w.recs.resize((size_t)std::max(r.m, 1));
        w.nrec = make_clause_records(r.clauses.data(), r.m, r.k, w.recs.data(), QNAE_PRED_NAE, &w.nlow);
        w.rec_at = B.take(sizeof(ClauseRec) * (size_t)std::max(w.nrec, 1));
        const int T = r.p > 0 ? r.p : 1;
        w.tabs.resize((size_t)T * (r.m + 1));
        w.forms.resize((size_t)T);
        r.final_scale = build_tables(r.n, r.m, r.gammas.data(), r.betas.data(), r.p, w.tabs.data(), w.forms.data());
        w.tab_at = B.take(r.part_off);  // same layout as the aux block: tables, then forms
        if (!r.resident) {
            plan_sweeps(r.plan, r.n, r.m, r.p, r.dtype, r.shape.tile_bits, r.shape.low_run_bits, r.shape.page_bit,
                        r.shape.split, false,
                        w.forms.data(), r.final_scale);
            r.plan.half = r.half;
        }
    }
    // Cost launches per cost type.
    std::vector<New*> cgroups[2];
    for (auto& w : nw) cgroups[w.r->dtype == QNAE_U16 ? 1 : 0].push_back(&w);
    size_t cargs_at[2], cfirst_at[2];
    for (int g = 0; g < 2; ++g) {
        cargs_at[g] = B.take(sizeof(qnae::CostArgs) * cgroups[g].size());
        cfirst_at[g] = B.take(sizeof(uint32_t) * (cgroups[g].size() + 1));
    }
    // Resident launches: new small requests run whole this tick.
    std::vector<New*> res[2];
    for (auto& w : nw)
        if (w.r->resident) res[w.r->dtype == QNAE_U16 ? 1 : 0].push_back(&w);
    size_t res_at[2];
    for (int g = 0; g < 2; ++g) res_at[g] = B.take(sizeof(qnae::ResidentArgs) * res[g].size());
    // Rounds of sweeps over the large requests.
    std::vector<Request*> large;
    size_t most = 0;
    double round_bytes = 0;
    for (Request* r : active)
        if (!r->resident) {
            large.push_back(r);
            most = std::max(most, r->plan.ops.size() - r->next_op);
            round_bytes += 17.0 * (double)(1ull << (r->n - (r->half ? 1 : 0)));
        }
    size_t rounds = most;
    if (round_bytes > 0) rounds = std::min(rounds, std::max<size_t>(1, (size_t)(tick_bytes / round_bytes)));
    struct Launch {
        int kind, dtype;
        bool half;
        int tb;
        std::vector<Request*> members;
        size_t args_at, first_at;
        uint32_t blocks;
    };
    std::vector<std::map<std::tuple<int, int, bool, int>, Launch>> sweeps(rounds);
    std::vector<Request*> finishing;
    for (Request* r : large) {
        for (size_t k = 0; k < rounds && r->next_op + k < r->plan.ops.size(); ++k) {
            const Op& op = r->plan.ops[r->next_op + k];
            Launch& L = sweeps[k][std::make_tuple(op.kind, r->dtype, r->half, r->shape.tile_bits)];
            L.kind = op.kind;
            L.dtype = r->dtype;
            L.half = r->half;
            L.tb = r->shape.tile_bits;
            L.members.push_back(r);
        }
        if (r->next_op + rounds >= r->plan.ops.size()) finishing.push_back(r);
    }
    for (auto& round : sweeps)
        for (auto& kv : round) {
            kv.second.args_at = B.take(sizeof(SweepArgs) * kv.second.members.size());
            kv.second.first_at = B.take(sizeof(uint32_t) * (kv.second.members.size() + 1));
        }
    const size_t rp_at = B.take(sizeof(double*) * finishing.size());
    const size_t rb_at = B.take(sizeof(uint32_t) * finishing.size());
    const size_t ro_at = B.take(sizeof(double*) * finishing.size());
    // Results of every request that ends this tick, gathered for one copy back.
    std::vector<Request*> done;
    for (int g = 0; g < 2; ++g)
        for (New* w : res[g]) done.push_back(w->r);
    for (Request* r : finishing) done.push_back(r);
    const size_t out_at = B.take(sizeof(double) * 3 * std::max<size_t>(done.size(), 1));
    if (admitted.empty() && large.empty()) return QNAE_OK;
    HIP_TRY(h_blob.reserve(B.size));
    HIP_TRY(d_blob.reserve(B.size));
    char* h = (char*)h_blob.ptr;
    char* d = (char*)d_blob.ptr;
    std::unordered_map<Request*, double*> out_of;
    for (size_t q = 0; q < done.size(); ++q) out_of[done[q]] = (double*)(d + out_at) + 3 * q;
    for (auto& w : nw) {
        std::memcpy(h + w.rec_at, w.recs.data(), sizeof(ClauseRec) * (size_t)w.nrec);
        std::memcpy(h + w.tab_at, w.tabs.data(), sizeof(float2) * w.tabs.size());
        std::memcpy(h + w.tab_at + w.r->form_off, w.forms.data(), sizeof(MixForm) * w.forms.size());
    }
    uint32_t cblocks[2] = {0, 0};
    int cmax[2] = {0, 0};
    bool cwide[2] = {false, false};  // some clause variable at index 32 or above
    for (int g = 0; g < 2; ++g) {
        qnae::CostArgs* args = (qnae::CostArgs*)(h + cargs_at[g]);
        uint32_t* first = (uint32_t*)(h + cfirst_at[g]);
        for (size_t q = 0; q < cgroups[g].size(); ++q) {
            const New& w = *cgroups[g][q];
            args[q].clauses = (const ClauseRec*)(d + w.rec_at);
            args[q].num_clauses = w.nrec;
            args[q].num_low = w.nlow;
            const int states = w.r->n - (w.r->half ? 1 : 0);  // half: the lower half of the diagonal
            args[q].n = states;
            args[q].cost = pool + w.r->cost_off;
            args[q].zeros = nullptr;
            first[q] = cblocks[g];
            cwide[g] = cwide[g] || w.r->n > 32;
            const uint64_t threads = states >= 5 ? (1ull << (states - 5)) : 1ull;
            cblocks[g] += (uint32_t)((threads + 255) / 256);
            cmax[g] = std::max(cmax[g], w.nrec);
        }
        first[cgroups[g].size()] = cblocks[g];
    }
    for (int g = 0; g < 2; ++g) {
        qnae::ResidentArgs* ra = (qnae::ResidentArgs*)(h + res_at[g]);
        for (size_t q = 0; q < res[g].size(); ++q) {
            const New& w = *res[g][q];
            const Request& r = *w.r;
            ra[q].state_in = nullptr;
            ra[q].cost = pool + r.cost_off;
            ra[q].luts = (const float2*)(d + w.tab_at);
            ra[q].forms = (const MixForm*)(d + w.tab_at + r.form_off);
            ra[q].state_out = nullptr;
            ra[q].out = out_of[w.r];
            ra[q].store_scale = make_float2(1.f, 0.f);
            ra[q].n = r.n;
            ra[q].p = r.p;
            ra[q].lut_len = r.m + 1;
        }
    }
    for (size_t k = 0; k < rounds; ++k)
        for (auto& kv : sweeps[k]) {
            Launch& L = kv.second;
            SweepArgs* args = (SweepArgs*)(h + L.args_at);
            uint32_t* first = (uint32_t*)(h + L.first_at);
            L.blocks = 0;
            for (size_t q = 0; q < L.members.size(); ++q) {
                Request& r = *L.members[q];
                char* aux = pool + r.aux_off;
                sweep_args(r.plan, r.plan.ops[r.next_op + k], (float2*)(pool + r.state_off), pool + r.cost_off,
                           (const float2*)aux, (double*)(aux + r.part_off), &args[q]);
                first[q] = L.blocks;
                L.blocks += r.tiles;
            }
            first[L.members.size()] = L.blocks;
        }
    {
        const double** rp = (const double**)(h + rp_at);
        uint32_t* rb = (uint32_t*)(h + rb_at);
        double** ro = (double**)(h + ro_at);
        for (size_t q = 0; q < finishing.size(); ++q) {
            Request& r = *finishing[q];
            rp[q] = (const double*)(pool + r.aux_off + r.part_off);
            rb[q] = r.tiles;
            ro[q] = out_of[&r];
        }
    }
    HIP_TRY(hipMemcpyAsync(d, h, B.size, hipMemcpyHostToDevice, s));
    for (auto& w : nw)
        if (!w.r->resident)
            HIP_TRY(hipMemcpyAsync(pool + w.r->aux_off, d + w.tab_at, w.r->part_off, hipMemcpyDeviceToDevice, s));
    for (int g = 0; g < 2; ++g) {
        if (cgroups[g].empty()) continue;
        HIP_TRY(qnae::launch_cost_batch((const qnae::CostArgs*)(d + cargs_at[g]), (const uint32_t*)(d + cfirst_at[g]),
                                        (int)cgroups[g].size(), cblocks[g], g ? QNAE_U16 : QNAE_U8, cmax[g], cwide[g], s));
        ++launches;
    }
    for (int g = 0; g < 2; ++g) {
        if (res[g].empty()) continue;
        HIP_TRY(qnae::launch_resident_batch(g ? QNAE_U16 : QNAE_U8, (const qnae::ResidentArgs*)(d + res_at[g]),
                                            (int)res[g].size(), s));
        ++launches;
    }
    for (size_t k = 0; k < rounds; ++k)
        for (auto& kv : sweeps[k]) {
            const Launch& L = kv.second;
            HIP_TRY(qnae::launch_sweep_batch(L.tb, L.dtype, L.kind, (const SweepArgs*)(d + L.args_at),
                                             (const uint32_t*)(d + L.first_at), (int)L.members.size(), L.blocks, s,
                                             L.half));
            ++launches;
        }
    if (!finishing.empty()) {
        HIP_TRY(qnae::launch_final_reduce_batch((const double* const*)(d + rp_at), (const uint32_t*)(d + rb_at),
                                                (double* const*)(d + ro_at), (int)finishing.size(), s));
        ++launches;
    }
    if (!done.empty())
        HIP_TRY(hipMemcpyAsync(h + out_at, d + out_at, sizeof(double) * 3 * done.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double t = now_s();
    const double* hres = (const double*)(h + out_at);
    {
        std::lock_guard<std::mutex> g(mu);
        for (Request* r : large) r->next_op = std::min(r->plan.ops.size(), r->next_op + rounds);
        for (size_t q = 0; q < done.size(); ++q) {
            Request& r = *done[q];
            const double sc = std::norm(r.final_scale) * (r.half ? 2.0 : 1.0);
            r.result.p_success = hres[3 * q] * sc;
            r.result.expected_cost = hres[3 * q + 1] * sc;
            r.result.norm = hres[3 * q + 2] * sc;
            r.t_done = t;
            r.state = r.cancel ? Request::CANCELED : Request::DONE;  // a cancel promised no result
            release(r);
            if (r.state == Request::DONE) ++completed;
        }
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [](Request* r) {
                                        return r->state == Request::DONE || r->state == Request::CANCELED;
                                    }),
                     active.end());
        ++ticks;
    }
    cv_done.notify_all();
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

void qnae_server::run() {
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Request*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (queue.empty() && active.empty() && stop) return;
            // cancelled active requests leave between ticks (no work of theirs is in flight)
            bool dropped = false;
            for (Request* r : active)
                if (r->cancel) {
                    r->state = Request::CANCELED;
                    release(*r);
                    dropped = true;
                }
            if (dropped) {
                active.erase(std::remove_if(active.begin(), active.end(),
                                            [](Request* r) { return r->state == Request::CANCELED; }),
                             active.end());
                cv_done.notify_all();
            }
            // FIFO admission while a slot and the pool allow it
            while (!queue.empty() && (int)active.size() < max_slots) {
                Request& r = *queue.front();
                int so, co, ao;
                plan_blocks(r, &so, &co, &ao);
                uint64_t soff = 0, coff = 0, aoff = 0;
                // largest block first: the state, then the cost, then the aux
                if (so >= 0 && !buddy->alloc(so, &soff)) break;
                if (!buddy->alloc(co, &coff)) {
                    if (so >= 0) buddy->release(soff, so);
                    break;
                }
                if (ao >= 0 && !buddy->alloc(ao, &aoff)) {
                    if (so >= 0) buddy->release(soff, so);
                    buddy->release(coff, co);
                    break;
                }
                r.cost_off = coff;
                r.cost_order = co;
                r.aux_off = aoff;
                r.aux_order = ao;
                r.state_off = soff;
                r.state_order = so;
                r.state = Request::ACTIVE;
                queue.pop_front();
                active.push_back(&r);
                admitted.push_back(&r);
            }
        }
        int rc;
        try {
            rc = tick(admitted);
        } catch (...) {  // host memory ran out inside the tick: fail like a device error
            rc = host_exception();
        }
        if (rc != QNAE_OK) {
            fail_server(this, rc);
            std::lock_guard<std::mutex> g(mu);
            for (Request* r : active) {
                r->state = Request::FAILED;
                release(*r);
            }
            active.clear();
            for (Request* r : queue) r->state = Request::FAILED;
            queue.clear();
            cv_done.notify_all();
            return;
        }
    }
}

extern "C" {

int qnae_server_create(qnae_ctx* ctx, uint64_t pool_bytes, int32_t max_slots, qnae_server** out) try {
    if (!out) return fail(QNAE_EINVAL, "null output pointer");
    *out = nullptr;
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    if (max_slots < 1 || max_slots > 65536) return fail(QNAE_EINVAL, "max_slots=%d outside [1, 65536]", max_slots);
    if (pool_bytes < (1ull << 20)) return fail(QNAE_EINVAL, "pool_bytes=%llu below 1 MiB", (unsigned long long)pool_bytes);
    int order = 63;
    while ((1ull << order) > pool_bytes) --order;
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<qnae_server> S(new qnae_server());
    S->ctx = ctx;
    S->device = ctx->device;
    S->tunes = ctx->tunes;
    S->default_shape = qnae_tune{ctx->tile_bits, ctx->min_low_run, ctx->page_bit, 0, 0.0};
    S->max_slots = max_slots;
    S->pool_bytes = 1ull << order;
    if (const char* e = std::getenv("QNAE_SERVER_HALF")) S->use_half = std::atoi(e) != 0;
    if (const char* e = std::getenv("QNAE_FAULT_INJECT"))
        if (std::strncmp(e, "server_tick:", 12) == 0) S->fault_tick = std::strtoull(e + 12, nullptr, 10);
    if (const char* e = std::getenv("QNAE_SERVER_TICK_BYTES")) S->tick_bytes = std::max(1.0, std::atof(e));
    S->buddy.reset(new Buddy(order));  // host allocations before the device ones
    HIP_TRY(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    hipError_t e = hipMalloc((void**)&S->pool, S->pool_bytes);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(S->stream);
        return fail(QNAE_ENOMEM, "server pool of %llu bytes: %s", (unsigned long long)S->pool_bytes, hipGetErrorString(e));
    }
    qnae_server* raw = S.release();
    try {
        raw->worker = std::thread([raw] { raw->run(); });
    } catch (...) {  // no scheduler thread: release what was allocated
        (void)hipFree(raw->pool);
        (void)hipStreamDestroy(raw->stream);
        delete raw;
        throw;
    }
    *out = raw;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_server_submit(qnae_server* S, const int32_t* clauses, int32_t m, int32_t n, int32_t k, const double* gammas,
                       const double* betas, int32_t p, uint64_t* ticket) try {
    if (!S || !ticket) return fail(QNAE_EINVAL, "null argument");
    const int dtype = m <= 255 ? QNAE_U8 : QNAE_U16;
    if (int rc = check_cost_args(n, m, dtype)) return rc;
    if (int rc = check_literals(clauses, m, n, k)) return rc;
    if (p < 0 || p > 100000) return fail(QNAE_EINVAL, "p=%d outside [0, 100000]", p);
    if (p > 0 && (!gammas || !betas)) return fail(QNAE_EINVAL, "null angle arrays with p=%d", p);
    for (int l = 0; l < p; ++l)
        if (!std::isfinite(gammas[l]) || !std::isfinite(betas[l]))
            return fail(QNAE_EINVAL, "non-finite angle at layer %d", l);
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->m = m;
    r->k = k;
    r->p = p;
    r->dtype = dtype;
    r->clauses.assign(clauses, clauses + (size_t)m * k);
    if (p > 0) {
        r->gammas.assign(gammas, gammas + p);
        r->betas.assign(betas, betas + p);
    }
    r->resident = n <= kResidentMaxN;
    r->half = !r->resident && S->use_half;
    {
        auto it = S->tunes.find({n, dtype});
        r->shape = it != S->tunes.end() ? it->second : S->default_shape;
    }
    r->tiles = r->resident ? 0u : 1u << (n - (r->half ? 1 : 0) - r->shape.tile_bits);
    int so, co, ao;
    if (!S->plan_blocks(*r, &so, &co, &ao))
        return fail(QNAE_EINVAL, "request with n=%d does not fit a pool of %llu bytes", n,
                    (unsigned long long)S->pool_bytes);
    std::lock_guard<std::mutex> g(S->mu);
    if (S->error != QNAE_OK) return fail(S->error, "server failed: %s", S->error_msg.c_str());
    if (S->stop) return fail(QNAE_EINVAL, "server is shutting down");
    if (S->queue.size() >= (1u << 20)) return fail(QNAE_EBUSY, "request queue full");
    r->ticket = S->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->all.emplace(r->ticket, std::move(r));
    S->cv_work.notify_one();
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_server_wait(qnae_server* S, uint64_t ticket, int32_t timeout_ms, qnae_result* out, double* latency_s) try {
    if (!S || !out) return fail(QNAE_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(QNAE_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    auto ready = [&] {
        return r->state == Request::DONE || r->state == Request::FAILED || r->state == Request::CANCELED;
    };
    if (timeout_ms < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return fail(QNAE_ETIMEDOUT, "ticket %llu not done", (unsigned long long)ticket);
    if (r->state == Request::CANCELED) {
        S->all.erase(it);
        return fail(QNAE_ECANCELED, "ticket %llu was cancelled", (unsigned long long)ticket);
    }
    if (r->state == Request::FAILED) {
        const std::string msg = S->error_msg;
        S->all.erase(it);
        return fail(QNAE_EHIP, "request failed: %s", msg.c_str());
    }
    *out = r->result;
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    S->all.erase(it);
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_server_cancel(qnae_server* S, uint64_t ticket) try {
    if (!S) return fail(QNAE_EINVAL, "null server");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(QNAE_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    switch (r->state) {
        case Request::DONE: return 1;
        case Request::QUEUED:
            S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), r), S->queue.end());
            r->state = Request::CANCELED;
            S->cv_done.notify_all();
            return QNAE_OK;
        case Request::ACTIVE:
            r->cancel = true;  // the scheduler drops it before its next tick
            S->cv_work.notify_one();
            return QNAE_OK;
        default: return QNAE_OK;  // failed or already cancelled: it will not complete
    }
} catch (...) {
    return host_exception();
}

int qnae_server_pool_in_use(qnae_server* S, uint64_t* bytes) try {
    if (!S || !bytes) return fail(QNAE_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(S->mu);
    *bytes = S->buddy->used();
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_server_stats(qnae_server* S, uint64_t* completed, uint64_t* ticks, uint64_t* launches,
                      uint64_t* peak_pool_bytes, uint64_t* queued, uint64_t* active) try {
    if (!S) return fail(QNAE_EINVAL, "null server");
    std::lock_guard<std::mutex> g(S->mu);
    if (completed) *completed = S->completed;
    if (ticks) *ticks = S->ticks;
    if (launches) *launches = S->launches;
    if (peak_pool_bytes) *peak_pool_bytes = S->buddy->peak();
    if (queued) *queued = S->queue.size();
    if (active) *active = S->active.size();
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_server_destroy(qnae_server* S) try {
    if (!S) return QNAE_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    (void)hipStreamSynchronize(S->stream);
    (void)hipFree(S->pool);
    S->d_blob.release();
    S->h_blob.release();
    (void)hipStreamDestroy(S->stream);
    delete S;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
