// Host-side checks of the sweep planner and the clause records of the cost
// kernel, built with AddressSanitizer and UBSan for the host (no GPU call).
// Exit status 0 when every check holds.
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <new>
#include <stdexcept>
#include <algorithm>
#include <vector>

#include "../../paper_2401_02852_amd/csrc/host.h"

using namespace qnae_host;

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);    \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// Every index bit is mixed by exactly one group; a tile has TB distinct bits
// below n whose lowest four are x bits 0..3; each layer of a plan mixes every
// group once, with the phase table of layer l between its mixings.
static void check_groups_and_plans() {
    std::vector<qnae::MixForm> forms(8, qnae::MixForm{0.5f, 0});
    for (int TB = 12; TB <= 14; ++TB)
        for (int cmin = 4; cmin <= 6; ++cmin)
            for (int page : {18, 64})
                for (int split = 0; split <= 3; ++split)
                for (int n = TB + 1; n <= 34; ++n) {
                    const std::vector<Group> g = make_groups(n, TB, cmin, page, split);
                    uint64_t mixed = 0;
                    for (const Group& gr : g) {
                        CHECK((int)gr.pos.size() == TB);
                        uint64_t seen = 0;
                        for (int i = 0; i < TB; ++i) {
                            CHECK(gr.pos[i] >= 0 && gr.pos[i] < n);
                            CHECK(!((seen >> gr.pos[i]) & 1u));
                            seen |= 1ull << gr.pos[i];
                            if (i < 4) CHECK(gr.pos[i] == i);
                            if ((gr.mask >> i) & 1u) {
                                CHECK(!((mixed >> gr.pos[i]) & 1u));
                                mixed |= 1ull << gr.pos[i];
                            }
                        }
                    }
                    CHECK(mixed == ((n == 64 ? 0ull : 1ull << n) - 1ull));
                    for (int p : {0, 1, 2, 5}) {
                        const std::vector<Op> ops = make_plan((int)g.size(), p);
                        std::vector<int> count((size_t)(p > 0 ? p : 1) * g.size(), 0);
                        for (const Op& op : ops) {
                            CHECK(op.group >= 0 && op.group < (int)g.size());
                            for (int l : {op.pre_layer, op.post_layer})
                                if (l >= 0) {
                                    CHECK(l < p);
                                    ++count[(size_t)l * g.size() + op.group];
                                }
                        }
                        if (p > 0)
                            for (int c : count) CHECK(c == 1);
                        // half-state sweeps: the tile index fills n-1-TB stored bits
                        if (n - 1 > TB && n >= 15) {
                            SweepPlan P;
                            plan_sweeps(P, n, 10, p, QNAE_U8, TB, cmin, page, split, false, forms.data(),
                                        std::complex<double>(1.0, 0.0));
                            P.half = true;
                            for (const Op& op : P.ops) {
                                qnae::SweepArgs a;
                                sweep_args(P, op, nullptr, nullptr, nullptr, nullptr, &a);
                                CHECK(a.half == 1 && a.nw == n - 1 - TB);
                                CHECK(popcount64(a.wmask) == n - 1 - TB);
                                CHECK((a.wmask >> (n - 1)) == 0ull && (a.wmask & a.tile_bits) == 0ull);
                                const Group& gr = P.groups[op.group];
                                bool has_top = false;
                                for (int i = 0; i < TB; ++i) has_top |= gr.pos[i] == n - 1;
                                CHECK(has_top == (a.vbit >= 0));
                                if (a.vbit >= 0) CHECK(gr.pos[a.vbit] == n - 1);
                                CHECK(a.mir == (1ull << (n - 1)) - 1ull);
                            }
                        }
                    }
                }
}

// The records' tables and masks reproduce the clause predicate at every
// position of a 32-state run, for random high bits (NAE and k-SAT).
static void check_clause_records() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 4000; ++trial) {
        const int n = 6 + (int)(rng() % 40), k = 1 + (int)(rng() % 6);
        std::vector<int32_t> cl(k);
        for (int j = 0; j < k; ++j) {
            const int v = 1 + (int)(rng() % n);
            cl[j] = (rng() & 1u) ? -v : v;
        }
        for (int pred : {QNAE_PRED_NAE, QNAE_PRED_SAT}) {
            qnae::ClauseRec r;
            const int nrec = make_clause_records(cl.data(), 1, k, &r, pred);
            for (int rep = 0; rep < 8; ++rep) {
                const uint64_t xhi = (rng() & ((n >= 64 ? ~0ull : (1ull << n) - 1ull))) & ~31ull;
                for (uint32_t j = 0; j < 32; ++j) {
                    const uint64_t x = xhi | j;
                    int ntrue = 0;
                    for (int q = 0; q < k; ++q) {
                        const int v = (cl[q] > 0 ? cl[q] : -cl[q]) - 1;
                        const int bit = (int)((x >> v) & 1u);
                        ntrue += cl[q] > 0 ? bit : 1 - bit;
                    }
                    const bool want = pred == QNAE_PRED_NAE ? (ntrue == 0 || ntrue == k) : ntrue == 0;
                    bool got = false;
                    if (nrec == 1) {
                        const uint32_t hlo = ((uint32_t)x ^ r.pat_lo) & r.mask_hi_lo;
                        const uint32_t hhi = ((uint32_t)(x >> 32) ^ r.pat_hi) & r.mask_hi_hi;
                        const bool none = (hlo | hhi) == 0u;
                        const bool all = hlo == r.mask_hi_lo && hhi == r.mask_hi_hi;
                        const uint32_t carry = (none ? r.zero_tab : 0u) | (all ? r.full_tab : 0u);
                        got = (carry >> j) & 1u;
                    }
                    CHECK(got == want);
                }
            }
        }
    }
}

// The host worker pool runs every index exactly once per run, across many
// runs of different sizes, and shuts down cleanly.
// Phase rows: scale * exp(sign i g c) through the two-level angle addition
// against a direct sine and cosine of g c per entry; both round to FP32 values
// that lie within 1e-10 of each other, so entries differ by at most one FP32
// rounding step.
static void check_phase_rows() {
    std::mt19937_64 rng(11);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (int m : {0, 1, 15, 16, 17, 255, 256, 257, 300, 4097, 65535})
        for (int sign : {-1, +1})
            for (int trial = 0; trial < 4; ++trial) {
                const double g = 7.0 * U(rng);
                const std::complex<double> scale(U(rng), U(rng));
                std::vector<float2> row((size_t)m + 1);
                phase_row(g, m, scale, sign, row.data());
                const double tol = 1.2e-7 * std::abs(scale) + 2e-10;
                for (int c = 0; c <= m; ++c) {
                    const std::complex<double> e =
                        scale * std::complex<double>(std::cos(g * c), sign * std::sin(g * c));
                    CHECK(std::fabs(row[c].x - e.real()) <= tol && std::fabs(row[c].y - e.imag()) <= tol);
                }
            }
}

static void check_worker_pool() {
    for (int workers : {1, 3, 7}) {
        qnae_host::WorkerPool pool(workers);
        for (int count : {0, 1, 2, 5, 64, 1000}) {
            for (int rep = 0; rep < 20; ++rep) {
                std::vector<std::atomic<int>> hits(count > 0 ? count : 1);
                for (auto& h : hits) h.store(0);
                pool.run(count, [&](int i) { hits[i].fetch_add(1); });
                for (int i = 0; i < count; ++i) CHECK(hits[i].load() == 1);
            }
        }
        // a throwing item: the caller sees the exception after every worker
        // is idle, no item runs twice, and the pool serves the next run
        for (int rep = 0; rep < 20; ++rep) {
            const int count = 500;
            std::vector<std::atomic<int>> hits(count);
            for (auto& h : hits) h.store(0);
            bool thrown = false;
            try {
                pool.run(count, [&](int i) {
                    hits[i].fetch_add(1);
                    if (i == 37 || i == 400) throw std::runtime_error("item failed");
                });
            } catch (const std::runtime_error&) {
                thrown = true;
            }
            CHECK(thrown);
            CHECK(hits[37].load() == 1);
            for (int i = 0; i < count; ++i) CHECK(hits[i].load() <= 1);
            std::vector<std::atomic<int>> again(64);
            for (auto& h : again) h.store(0);
            pool.run(64, [&](int i) { again[i].fetch_add(1); });
            for (int i = 0; i < 64; ++i) CHECK(again[i].load() == 1);
        }
    }
}

// Entry points end in a catch-all that turns the exception being handled
// into a status code and this thread's last error.
static void check_host_exception() {
    int rc = 0;
    try {
        throw std::bad_alloc();
    } catch (...) {
        rc = host_exception();
    }
    CHECK(rc == QNAE_ENOMEM && std::string(last_error()).find("allocation") != std::string::npos);
    try {
        throw std::runtime_error("thread limit");
    } catch (...) {
        rc = host_exception();
    }
    CHECK(rc == QNAE_ENOMEM && std::string(last_error()).find("thread limit") != std::string::npos);
    try {
        throw 7;
    } catch (...) {
        rc = host_exception();
    }
    CHECK(rc == QNAE_ENOMEM && std::string(last_error()).find("unknown") != std::string::npos);
}

// The planner as first written with growable vectors (kept here as the
// reference for the fixed-storage planner the library uses, which must give
// the same groups and the same sweeps).
static std::vector<Group> vector_make_groups(int n, int TB, int cmin, int page) {
    std::vector<Group> g;
    Group A;
    if (n <= TB) {
        for (int i = 0; i < TB; ++i) A.pos.push_back(i);
        A.mask = (1u << TB) - 1u;
        g.push_back(A);
        return g;
    }
    const int rest = n - TB;
    const int h = (rest + (TB - cmin) - 1) / (TB - cmin);
    std::vector<int> P;
    for (int b = std::max(page, TB); b < n; ++b) P.push_back(b);
    const int target = ((int)P.size() + h) / (h + 1);
    const int a = std::min(std::min(target, TB - cmin), (int)P.size());
    const int cA = TB - a;
    std::vector<int> apage(P.end() - a, P.end());
    for (int i = 0; i < cA; ++i) A.pos.push_back(i);
    for (int b : apage) A.pos.push_back(b);
    A.mask = (1u << TB) - 1u;
    g.push_back(A);
    // bits left for the other groups, page bits first
    std::vector<int> RP, RN;
    for (int b = cA; b < n; ++b) {
        if (std::find(apage.begin(), apage.end(), b) != apage.end()) continue;
        (b >= page ? RP : RN).push_back(b);
    }
    const int R = (int)(RP.size() + RN.size());
    std::vector<std::vector<int>> piece(h);
    std::vector<int> size(h);
    for (int i = 0; i < h; ++i) size[i] = R / h + (i < R % h ? 1 : 0);
    for (int i = 0, q = (int)RP.size(); i < h; ++i) {  // consecutive page runs, evenly, top run first
        const int c = (int)RP.size() / h + (i < (int)RP.size() % h ? 1 : 0);
        q -= c;
        for (int k = 0; k < c; ++k) piece[i].push_back(RP[q + k]);
    }
    size_t nx = 0;
    for (int i = 0; i < h; ++i)
        while ((int)piece[i].size() < size[i]) piece[i].push_back(RN[nx++]);
    for (int i = 0; i < h; ++i) {
        Group B;
        std::vector<int> bits = piece[i];
        // fill up to TB - cmin bits with unmixed bits just above the low run
        std::vector<int> fill;
        for (int b = cmin; (int)(bits.size() + fill.size()) < TB - cmin; ++b)
            if (std::find(bits.begin(), bits.end(), b) == bits.end()) fill.push_back(b);
        std::vector<int> all = fill;
        all.insert(all.end(), bits.begin(), bits.end());
        std::sort(all.begin(), all.end());
        for (int b = 0; b < cmin; ++b) B.pos.push_back(b);
        B.mask = 0u;
        for (int b : all) {
            if (std::find(bits.begin(), bits.end(), b) != bits.end()) B.mask |= 1u << B.pos.size();
            B.pos.push_back(b);
        }
        g.push_back(B);
    }
    return g;
}

static std::vector<Op> vector_make_plan(int ngroups, int p, bool from_state) {
    using namespace qnae;
    std::vector<Op> ops;
    if (p == 0) {
        ops.push_back({0, SK_P0, -1, -1, 0});
        return ops;
    }
    // from a given state: load, phase 0, mix group 0 (a boundary sweep with
    // nothing to mix before the phase)
    ops.push_back(from_state ? Op{0, SK_BOUNDARY, -1, 0, 0} : Op{0, SK_FIRST, -1, 0, 0});
    std::vector<int> pending;  // groups not yet mixed for layer l
    for (int g = 1; g < ngroups; ++g) pending.push_back(g);
    for (int l = 0;; ++l) {
        if (pending.empty()) {  // one group: the previous sweep mixed it already
            if (l == p - 1) {
                ops.push_back({0, SK_FINAL, -1, -1, -1});
                return ops;
            }
            ops.push_back({0, SK_BOUNDARY, -1, l + 1, l + 1});
            continue;
        }
        int last = pending.back();
        for (int g : pending)
            if (g != 0) last = g;
        for (int g : pending)
            if (g != last) ops.push_back({g, SK_MIDDLE, l, -1, -1});
        if (l == p - 1) {
            ops.push_back({last, SK_FINAL, l, -1, -1});
            return ops;
        }
        ops.push_back({last, SK_BOUNDARY, l, l + 1, l + 1});
        pending.clear();
        for (int g = 0; g < ngroups; ++g)
            if (g != last) pending.push_back(g);
    }
}

// Half-state addressing as the sweep kernels compute it: every stored index
// y < 2^(n-1) is reached by exactly one element of one tile per sweep, for
// every tile shape, including tiles as large as the stored half (n - 1 = TB).
static void check_half_addressing() {
    std::vector<qnae::MixForm> forms(2, qnae::MixForm{0.5f, 0});
    for (int TB = 12; TB <= 14; ++TB)
        for (int cmin = 4; cmin <= 6; ++cmin)
            for (int page : {13, 64})
                for (int n = std::max(15, TB + 1); n <= 17; ++n) {
                    SweepPlan P;
                    plan_sweeps(P, n, 10, 2, QNAE_U8, TB, cmin, page, 0, false, forms.data(),
                                std::complex<double>(1.0, 0.0));
                    P.half = true;
                    const uint64_t N = 1ull << (n - 1);
                    std::vector<uint8_t> hits(N);
                    for (const Op& op : P.ops) {
                        qnae::SweepArgs a;
                        sweep_args(P, op, nullptr, nullptr, nullptr, nullptr, &a);
                        CHECK(a.nw == n - 1 - TB && popcount64(a.wmask) == a.nw);
                        std::fill(hits.begin(), hits.end(), 0);
                        for (uint64_t t = 0; t < (1ull << a.nw); ++t) {
                            uint64_t base = 0, w = t;
                            for (uint64_t m = a.wmask; m != 0ull; m &= m - 1ull, w >>= 1)
                                if (w & 1ull) base |= m & (~m + 1ull);
                            for (uint32_t e = 0; e < (1u << TB); ++e) {
                                uint64_t x = 0;
                                bool mirrored = false;
                                for (int i = 0; i < TB; ++i) {
                                    if (!((e >> i) & 1u)) continue;
                                    if (i == a.vbit) mirrored = true;
                                    else x |= 1ull << a.pos[i];
                                }
                                const uint64_t y = mirrored ? a.mir - (base + x) : base + x;
                                CHECK(y < N);
                                CHECK(hits[y] == 0);
                                hits[y] = 1;
                                // pairs along tile bit 0 are 16-byte aligned (mirrored ones one slot lower)
                                if (!(e & 1u)) CHECK(((mirrored ? y - 1 : y) & 1ull) == 0ull);
                            }
                        }
                        for (uint64_t y = 0; y < N; ++y) CHECK(hits[y] == 1);
                    }
                }
}

static void check_fixed_planner_matches_vectors() {
    for (int TB = 12; TB <= 14; ++TB)
        for (int cmin = 4; cmin <= 6; ++cmin)
            for (int page : {4, 13, 18, 22, 64})
                for (int n = TB + 1; n <= 34; ++n) {
                    const std::vector<Group> want = vector_make_groups(n, TB, cmin, page);
                    GroupSpec spec[kMaxGroups];
                    const int count = make_group_specs(n, TB, cmin, page, 0, spec);
                    CHECK(count == (int)want.size() && count <= kMaxGroups);
                    for (int i = 0; i < count; ++i) {
                        CHECK(spec[i].mask == want[i].mask);
                        for (int j = 0; j < TB; ++j) CHECK(spec[i].pos[j] == want[i].pos[j]);
                    }
                    for (int p : {0, 1, 2, 3, 7})
                        for (bool from_state : {false, true}) {
                            const std::vector<Op> a = vector_make_plan(count, p, from_state);
                            const std::vector<Op> b = make_plan(count, p, from_state);
                            CHECK(a.size() == b.size());
                            for (size_t q = 0; q < a.size(); ++q)
                                CHECK(a[q].group == b[q].group && a[q].kind == b[q].kind &&
                                      a[q].pre_layer == b[q].pre_layer && a[q].post_layer == b[q].post_layer &&
                                      a[q].lut_layer == b[q].lut_layer);
                        }
                }
}

// The split variants at the sizes where they were measured fastest: the
// index bits below the page bits that the third group mixes.
static uint64_t third_group_low_bits(int n, int split) {
    GroupSpec spec[kMaxGroups];
    CHECK(make_group_specs(n, 13, 4, 18, split, spec) == 3);
    uint64_t bits = 0;
    for (int i = 0; i < 13; ++i)
        if (((spec[2].mask >> i) & 1u) && spec[2].pos[i] < 18) bits |= 1ull << spec[2].pos[i];
    return bits;
}

static void check_split_layouts() {
    auto set = [](std::initializer_list<int> b) {
        uint64_t v = 0;
        for (int x : b) v |= 1ull << x;
        return v;
    };
    CHECK(third_group_low_bits(30, 0) == set({14, 15, 16, 17}));
    CHECK(third_group_low_bits(30, 1) == set({10, 15, 16, 17}));
    CHECK(third_group_low_bits(29, 2) == set({9, 14, 15, 16, 17}));
    CHECK(third_group_low_bits(31, 3) == set({8, 10, 15, 16, 17}));
    // a split changes nothing where there is no third group
    for (int n : {15, 20, 32, 33})
        for (int split = 1; split <= 3; ++split) {
            GroupSpec a[kMaxGroups], b[kMaxGroups];
            const int ca = make_group_specs(n, 13, 4, 18, 0, a), cb = make_group_specs(n, 13, 4, 18, split, b);
            CHECK(ca == cb);
            if (ca == 3) continue;
            for (int i = 0; i < ca; ++i) {
                CHECK(a[i].mask == b[i].mask);
                for (int j = 0; j < 13; ++j) CHECK(a[i].pos[j] == b[i].pos[j]);
            }
        }
}

// Records of clauses with a variable below 5 come first (num_low of them),
// each part in input order; a record on higher variables only has the
// all-ones zero table, the kernel's test for the constant part.
static void check_record_order() {
    std::mt19937_64 rng(11);
    for (int trial = 0; trial < 500; ++trial) {
        const int n = 6 + (int)(rng() % 40), k = 1 + (int)(rng() % 5), m = (int)(rng() % 60);
        std::vector<int32_t> cl((size_t)m * k);
        for (auto& l : cl) {
            const int v = 1 + (int)(rng() % n);
            l = (rng() & 1u) ? -v : v;
        }
        for (int pred : {QNAE_PRED_NAE, QNAE_PRED_SAT}) {
            std::vector<qnae::ClauseRec> recs((size_t)std::max(m, 1)), one(1);
            int nlow = -1;
            const int nrec = make_clause_records(cl.data(), m, k, recs.data(), pred, &nlow);
            CHECK(nlow >= 0 && nlow <= nrec);
            // the same records, one clause at a time in input order
            std::vector<qnae::ClauseRec> lo, hi;
            for (int i = 0; i < m; ++i) {
                if (make_clause_records(cl.data() + (size_t)i * k, 1, k, one.data(), pred) != 1) continue;
                bool low = false;
                for (int j = 0; j < k; ++j) low = low || (cl[(size_t)i * k + j] > 0 ? cl[(size_t)i * k + j]
                                                                                    : -cl[(size_t)i * k + j]) <= 5;
                (low ? lo : hi).push_back(one[0]);
                CHECK((one[0].zero_tab != ~0u) == low);
            }
            CHECK((int)lo.size() == nlow && (int)(lo.size() + hi.size()) == nrec);
            for (int i = 0; i < nrec; ++i) {
                const qnae::ClauseRec& want = i < nlow ? lo[(size_t)i] : hi[(size_t)(i - nlow)];
                CHECK(std::memcmp(&recs[(size_t)i], &want, sizeof want) == 0);
            }
        }
    }
}

int main() {
    check_fixed_planner_matches_vectors();
    check_half_addressing();
    check_groups_and_plans();
    check_split_layouts();
    check_clause_records();
    check_record_order();
    check_phase_rows();
    check_host_exception();
    check_worker_pool();
    std::printf("planner and clause records ok\n");
    return 0;
}
