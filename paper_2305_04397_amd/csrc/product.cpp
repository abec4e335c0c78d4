// Agent-task product MDPs M_i (x) A_j (Sec. 2, "Product MDP"; Sec. 3.1) built
// on the host, validated, concatenated with global indices and uploaded.
//
// Semantics: a product state (s, q) is done when q is accepting or a trap (a
// location from which no run reaches an accepting one).  Done states are
// absorbing with value 0 and are not stored; a row keeps its entries into
// live states, flags whether it moves mass into done, and carries the rewards
// (-cost(s, a), sum of P(s, a, s') over s' whose next location accepts).  Live
// reachable states are explored from (s0, q0) and numbered in (q, s) order.
#include "common.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <cmath>
#include <thread>
#include <unordered_map>

namespace morap {

namespace {

struct Built {
    int32_t init = -1;
    std::vector<int32_t> state_row{0}, row_ptr{0}, col, states_sq;
    std::vector<double> prob, rew;
    std::vector<uint8_t> to_done;
};

void validate_agent(const morap_agent& a, int i) {
    const std::string who = "agent " + std::to_string(i) + ": ";
    MORAP_CHECK(a.n_states > 0 && a.n_actions > 0 && a.n_actions <= 32, MORAP_E_INVALID,
                who + "need n_states > 0 and 0 < n_actions <= 32");
    MORAP_CHECK(a.init >= 0 && a.init < a.n_states, MORAP_E_INVALID, who + "init out of range");
    MORAP_CHECK(a.sa_ptr && a.cost, MORAP_E_INVALID, who + "NULL arrays");
    const int64_t rows = (int64_t)a.n_states * a.n_actions;
    MORAP_CHECK(a.sa_ptr[0] == 0, MORAP_E_INVALID, who + "sa_ptr[0] must be 0");
    for (int s = 0; s < a.n_states; ++s) {
        bool any = false;
        for (int act = 0; act < a.n_actions; ++act) {
            const int64_t r = (int64_t)s * a.n_actions + act;
            any |= a.sa_ptr[r + 1] > a.sa_ptr[r];
        }
        MORAP_CHECK(any, MORAP_E_INVALID, who + "a state without enabled actions");
    }
    for (int64_t r = 0; r < rows; ++r) {
        MORAP_CHECK(a.sa_ptr[r + 1] >= a.sa_ptr[r], MORAP_E_INVALID, who + "sa_ptr not monotone");
        MORAP_CHECK(std::isfinite(a.cost[r]), MORAP_E_INVALID, who + "non-finite cost");
        if (a.sa_ptr[r + 1] == a.sa_ptr[r]) continue;
        double sum = 0;
        for (int32_t e = a.sa_ptr[r]; e < a.sa_ptr[r + 1]; ++e) {
            MORAP_CHECK(a.succ[e] >= 0 && a.succ[e] < a.n_states, MORAP_E_INVALID, who + "successor out of range");
            MORAP_CHECK(std::isfinite(a.prob[e]) && a.prob[e] >= 0, MORAP_E_INVALID, who + "bad probability");
            sum += a.prob[e];
        }
        MORAP_CHECK(std::fabs(sum - 1.0) <= 1e-9, MORAP_E_INVALID,
                    who + "an enabled action's probabilities do not sum to 1");
    }
}

void validate_dfa(const morap_dfa& t, int j) {
    const std::string who = "task " + std::to_string(j) + ": ";
    MORAP_CHECK(t.n_locs > 0 && t.n_letters > 0, MORAP_E_INVALID, who + "empty automaton");
    MORAP_CHECK(t.q0 >= 0 && t.q0 < t.n_locs, MORAP_E_INVALID, who + "q0 out of range");
    MORAP_CHECK(t.delta && t.accepting, MORAP_E_INVALID, who + "NULL arrays");
    for (int64_t i = 0; i < (int64_t)t.n_locs * t.n_letters; ++i)
        MORAP_CHECK(t.delta[i] >= 0 && t.delta[i] < t.n_locs, MORAP_E_INVALID, who + "delta out of range");
}

// done locations: accepting, or no run reaches an accepting location
std::vector<uint8_t> done_locations(const morap_dfa& t) {
    std::vector<uint8_t> reach(t.n_locs, 0);
    for (int q = 0; q < t.n_locs; ++q) reach[q] = t.accepting[q] ? 1 : 0;
    for (bool changed = true; changed;) {
        changed = false;
        for (int q = 0; q < t.n_locs; ++q) {
            if (reach[q]) continue;
            for (int l = 0; l < t.n_letters; ++l)
                if (reach[t.delta[(int64_t)q * t.n_letters + l]]) {
                    reach[q] = 1;
                    changed = true;
                    break;
                }
        }
    }
    std::vector<uint8_t> done(t.n_locs);
    for (int q = 0; q < t.n_locs; ++q) done[q] = (t.accepting[q] || !reach[q]) ? 1 : 0;
    return done;
}

Built build_one(const morap_agent& a, const morap_dfa& t, const int32_t* letters) {
    Built b;
    const int S = a.n_states, Q = t.n_locs, L = t.n_letters, A = a.n_actions;
    const auto done = done_locations(t);
    auto next_loc = [&](int q, int s2) { return t.delta[(int64_t)q * L + letters[s2]]; };
    if (done[t.q0]) return b;   // nothing live: value 0
    // reachability over live states (dense (q, s) index)
    std::vector<int32_t> idx((size_t)S * Q, -1);
    std::vector<int32_t> stack;
    auto key = [&](int s, int q) { return (size_t)q * S + s; };
    idx[key(a.init, t.q0)] = 0;
    stack.push_back((int32_t)key(a.init, t.q0));
    while (!stack.empty()) {
        const size_t kq = (size_t)stack.back();
        stack.pop_back();
        const int q = (int)(kq / S), s = (int)(kq % S);
        for (int act = 0; act < A; ++act) {
            const int64_t r = (int64_t)s * A + act;
            for (int32_t e = a.sa_ptr[r]; e < a.sa_ptr[r + 1]; ++e) {
                const int s2 = a.succ[e];
                const int q2 = next_loc(q, s2);
                if (done[q2]) continue;
                const size_t k2 = key(s2, q2);
                if (idx[k2] < 0) {
                    idx[k2] = 0;
                    stack.push_back((int32_t)k2);
                }
            }
        }
    }
    // number the live states in (q, s) order
    int32_t n = 0;
    for (size_t kq = 0; kq < idx.size(); ++kq)
        if (idx[kq] >= 0) idx[kq] = n++;
    b.states_sq.reserve((size_t)2 * n);
    for (size_t kq = 0; kq < idx.size(); ++kq) {
        if (idx[kq] < 0) continue;
        const int q = (int)(kq / S), s = (int)(kq % S);
        b.states_sq.push_back(s);
        b.states_sq.push_back(q);
        for (int act = 0; act < A; ++act) {
            const int64_t r = (int64_t)s * A + act;
            if (a.sa_ptr[r + 1] == a.sa_ptr[r]) continue;   // disabled action
            double mass_acc = 0.0;
            uint8_t hits_done = 0;
            for (int32_t e = a.sa_ptr[r]; e < a.sa_ptr[r + 1]; ++e) {
                const int s2 = a.succ[e];
                const int q2 = next_loc(q, s2);
                if (done[q2]) {
                    hits_done = 1;
                    if (t.accepting[q2]) mass_acc += a.prob[e];
                } else {
                    b.col.push_back(idx[key(s2, q2)]);
                    b.prob.push_back(a.prob[e]);
                }
            }
            b.rew.push_back(-a.cost[r]);
            b.rew.push_back(mass_acc);
            b.to_done.push_back(hits_done);
            b.row_ptr.push_back((int32_t)b.col.size());
        }
        b.state_row.push_back((int32_t)b.to_done.size());
    }
    b.init = idx[key(a.init, t.q0)];
    return b;
}

}  // namespace

void check_agent(const morap_agent& a, int i) { validate_agent(a, i); }
void check_dfa(const morap_dfa& t, int j) { validate_dfa(t, j); }
std::vector<uint8_t> dfa_done(const morap_dfa& t) { return done_locations(t); }

static void concat(morap_ctx* c, std::vector<Built>& parts, int nI, int nJ) {
    HostModels hm;
    hm.nI = nI;
    hm.nJ = nJ;
    hm.M = nI * nJ;
    int64_t S = 0, R = 0, N = 0;
    for (auto& b : parts) {
        S += (int64_t)b.state_row.size() - 1;
        R += (int64_t)b.row_ptr.size() - 1;
        N += (int64_t)b.col.size();
    }
    const int64_t lim = 2147483647;
    MORAP_CHECK(S < lim && R < lim && N < lim, MORAP_E_UNSUPPORTED, "more than 2^31-1 states, rows or entries");
    hm.state_base.resize(hm.M + 1);
    hm.init.resize(hm.M);
    hm.state_row.reserve(S + 1);
    hm.row_ptr.reserve(R + 1);
    hm.col.reserve(N);
    hm.prob.reserve(N);
    hm.rew.reserve(2 * R);
    hm.to_done.reserve(R);
    hm.states_sq.reserve(2 * S);
    hm.state_row.push_back(0);
    hm.row_ptr.push_back(0);
    int max_rows = 0;
    for (int m = 0; m < hm.M; ++m) {
        Built& b = parts[m];
        const int32_t sb = (int32_t)(hm.state_row.size() - 1);
        const int32_t rb = (int32_t)(hm.row_ptr.size() - 1);
        const int32_t eb = (int32_t)hm.col.size();
        hm.state_base[m] = sb;
        hm.init[m] = b.init >= 0 ? sb + b.init : -1;
        for (size_t s = 1; s < b.state_row.size(); ++s) {
            hm.state_row.push_back(rb + b.state_row[s]);
            max_rows = std::max(max_rows, b.state_row[s] - b.state_row[s - 1]);
        }
        for (size_t r = 1; r < b.row_ptr.size(); ++r) hm.row_ptr.push_back(eb + b.row_ptr[r]);
        for (int32_t x : b.col) hm.col.push_back(sb + x);
        hm.prob.insert(hm.prob.end(), b.prob.begin(), b.prob.end());
        hm.rew.insert(hm.rew.end(), b.rew.begin(), b.rew.end());
        hm.to_done.insert(hm.to_done.end(), b.to_done.begin(), b.to_done.end());
        hm.states_sq.insert(hm.states_sq.end(), b.states_sq.begin(), b.states_sq.end());
        b = Built();   // free as we go
    }
    hm.state_base[hm.M] = (int32_t)(hm.state_row.size() - 1);
    MORAP_CHECK(max_rows <= 32, MORAP_E_UNSUPPORTED, "more than 32 rows in a state");
    c->hm = std::move(hm);
    c->max_rows_per_state = max_rows;
}

// Connected regions of at most HALO_TILE states of every agent's transition
// graph (edges from each state to its successor slots, both directions):
// seeds are taken in breadth-first order of the whole graph and each region
// grows breadth-first over unassigned states, so regions are compact and
// consecutive regions are neighbours.  reg[s] = region of s, pos[s] = its
// place in the region's growth order.
static void agent_regions(int64_t n, const int32_t* slot, std::vector<int32_t>& reg, std::vector<int32_t>& pos) {
    constexpr int NS = 5;
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t s = 0; s < n; ++s)
        for (int d = 1; d < NS; ++d) {
            const int32_t t = slot[s * NS + d];
            if (t >= 0 && t != s) {
                ++deg[s + 1];
                ++deg[t + 1];
            }
        }
    for (int64_t s = 0; s < n; ++s) deg[s + 1] += deg[s];
    std::vector<int32_t> adj(deg[n]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t s = 0; s < n; ++s)
        for (int d = 1; d < NS; ++d) {
            const int32_t t = slot[s * NS + d];
            if (t >= 0 && t != s) {
                adj[fill[s]++] = t;
                adj[fill[t]++] = (int32_t)s;
            }
        }
    // breadth-first order of the whole graph (every component)
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<uint8_t> seen(n, 0);
    for (int64_t r0 = 0; r0 < n; ++r0) {
        if (seen[r0]) continue;
        seen[r0] = 1;
        size_t head = order.size();
        order.push_back((int32_t)r0);
        while (head < order.size()) {
            const int32_t s = order[head++];
            for (int64_t e = deg[s]; e < deg[s + 1]; ++e)
                if (!seen[adj[e]]) {
                    seen[adj[e]] = 1;
                    order.push_back(adj[e]);
                }
        }
    }
    reg.assign(n, -1);
    pos.assign(n, 0);
    std::vector<int32_t> cur;
    int32_t nreg = 0;
    for (const int32_t seed : order) {
        if (reg[seed] >= 0) continue;
        cur.clear();
        cur.push_back(seed);
        reg[seed] = nreg;
        for (size_t head = 0; head < cur.size() && (int)cur.size() < HALO_TILE; ++head) {
            const int32_t s = cur[head];
            for (int64_t e = deg[s]; e < deg[s + 1] && (int)cur.size() < HALO_TILE; ++e)
                if (reg[adj[e]] < 0) {
                    reg[adj[e]] = nreg;
                    cur.push_back(adj[e]);
                }
        }
        for (size_t k = 0; k < cur.size(); ++k) pos[cur[k]] = (int32_t)k;
        ++nreg;
    }
}

// Halo tiles of the LDS-staged sweep (see its kernel), from the product
// states' block records (recs[8 g ..], in state order).  Per model, states are
// grouped by (location, agent region) in region order; groups are packed into
// tiles of at most HALO_TILE states and HALO_MAX halo rows, a group that
// alone exceeds the halo limit being halved.  Not built when a block index
// does not fit the record's 19 bits.
static void build_halo(HostModels& hm, const std::vector<int64_t>& abase, const std::vector<int32_t>& slot, int nI,
                       int nJ, const std::vector<int32_t>& recs, int64_t n_blocks) {
    hm.hal_tile.clear();
    hm.hal_tile_base.clear();
    hm.hal_list.clear();
    hm.hal_rec.clear();
    if (n_blocks >= (int64_t)1 << 19) return;
    constexpr int NS = 5;
    const int M = hm.M;
    const int32_t S = (int32_t)hm.S();
    std::vector<std::vector<int32_t>> reg(nI), pos(nI);
    {
        std::atomic<int> next{0};
        auto worker = [&] {
            for (int i; (i = next++) < nI;)
                agent_regions(abase[i + 1] - abase[i], &slot[(size_t)abase[i] * NS], reg[i], pos[i]);
        };
        const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (int k = 0; k < nt; ++k) th.emplace_back(worker);
        for (auto& k : th) k.join();
    }
    struct Part {
        std::vector<int32_t> tiles;   // model, rec_begin, n | H << 16, local halo begin
        std::vector<uint32_t> rec;
        std::vector<int32_t> list;
    };
    std::vector<Part> parts(M);
    std::atomic<int> next{0};
    auto worker = [&] {
        std::vector<int64_t> key;
        std::vector<int32_t> ord, stamp, place, own, halo, added;
        for (int m; (m = next++) < M;) {
            const int i = m / nJ;
            const int32_t s0 = hm.state_base[m], s1 = hm.state_base[m + 1], n = s1 - s0;
            if (n == 0) continue;
            Part& P = parts[m];
            // states sorted by (location, region, place in region)
            const int64_t nreg = (int64_t)abase[i + 1] - abase[i];
            key.resize(n);
            ord.resize(n);
            for (int32_t g = s0; g < s1; ++g) {
                const int32_t s = hm.states_sq[2 * (size_t)g], q = hm.states_sq[2 * (size_t)g + 1];
                key[g - s0] = ((int64_t)q * nreg + reg[i][s]) * HALO_TILE + pos[i][s];
                ord[g - s0] = g - s0;
            }
            std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
            stamp.assign(n, -1);
            place.assign(n, -1);
            int32_t tile_id = 0;
            own.clear();
            halo.clear();
            // rows a state brings: itself and its live successors (local)
            auto rows_of = [&](int32_t l, int32_t* out) {
                int k = 0;
                out[k++] = l;
                for (int d = 0; d < NS; ++d) {
                    const int32_t r = recs[(size_t)(s0 + l) * 8 + d];
                    if (r != S) out[k++] = r - s0;
                }
                return k;
            };
            // try to add states ord[b..e) to the open tile; false (and nothing
            // changed) when a limit would be exceeded
            auto try_add = [&](size_t b, size_t e) {
                if (own.size() + (e - b) > (size_t)HALO_TILE) return false;
                added.clear();
                int32_t rr[NS + 1];
                for (size_t p = b; p < e; ++p) {
                    const int k = rows_of(ord[p], rr);
                    for (int z = 0; z < k; ++z)
                        if (stamp[rr[z]] != tile_id) {
                            stamp[rr[z]] = tile_id;
                            added.push_back(rr[z]);
                        }
                }
                if (halo.size() + added.size() > (size_t)HALO_MAX) {
                    for (int32_t l : added) stamp[l] = -1;
                    return false;
                }
                for (size_t p = b; p < e; ++p) own.push_back(ord[p]);
                halo.insert(halo.end(), added.begin(), added.end());
                return true;
            };
            auto close = [&] {
                if (own.empty()) return;
                const int32_t hb = (int32_t)P.list.size();
                const int32_t rb = s0 + (int32_t)(P.rec.size() / 2);
                // halo list: own states first (record order), then the rest
                int32_t h = 0;
                for (int32_t l : own) {
                    place[l] = h++;
                    P.list.push_back(s0 + l);
                }
                for (int32_t l : halo)
                    if (place[l] < 0) {   // not one of the own states
                        place[l] = h++;
                        P.list.push_back(s0 + l);
                    }
                for (int32_t l : own) {
                    const int32_t* r = &recs[(size_t)(s0 + l) * 8];
                    uint32_t loc[NS];
                    for (int d = 0; d < NS; ++d) loc[d] = r[d] == S ? (uint32_t)HALO_MAX : (uint32_t)place[r[d] - s0];
                    P.rec.push_back(loc[0] | loc[1] << 8 | loc[2] << 16 | loc[3] << 24);
                    P.rec.push_back(loc[4] | ((uint32_t)r[6] & 31u) << 8 | (uint32_t)r[5] << 13);
                }
                P.tiles.insert(P.tiles.end(), {m, rb, (int32_t)own.size() | h << 16, hb});
                for (int32_t l : halo) place[l] = -1;
                for (int32_t l : own) place[l] = -1;
                own.clear();
                halo.clear();
                ++tile_id;
            };
            // add [b, e) to the open tile, else to a fresh one, else halve it
            std::function<void(size_t, size_t)> put = [&](size_t b, size_t e) {
                if (try_add(b, e)) return;
                close();
                if (try_add(b, e)) return;
                const size_t mid = b + (e - b) / 2;
                put(b, mid);
                put(mid, e);
            };
            for (size_t b = 0; b < (size_t)n;) {
                size_t e = b + 1;
                while (e < (size_t)n && key[ord[e]] / HALO_TILE == key[ord[b]] / HALO_TILE) ++e;
                put(b, e);
                b = e;
            }
            close();
        }
    };
    const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k) th.emplace_back(worker);
    for (auto& k : th) k.join();
    hm.hal_tile_base.assign(M + 1, 0);
    size_t nl = 0;
    for (int m = 0; m < M; ++m) nl += parts[m].list.size();
    MORAP_CHECK(nl < (size_t)0x7fffffff, MORAP_E_UNSUPPORTED, "halo lists exceed 2^31 entries");
    hm.hal_rec.resize((size_t)2 * S);
    hm.hal_list.reserve(nl);
    for (int m = 0; m < M; ++m) {
        Part& P = parts[m];
        hm.hal_tile_base[m] = (int32_t)(hm.hal_tile.size() / 4);
        const int32_t lb = (int32_t)hm.hal_list.size();
        for (size_t t = 0; t < P.tiles.size(); t += 4) {
            hm.hal_tile.insert(hm.hal_tile.end(), {P.tiles[t], P.tiles[t + 1], P.tiles[t + 2], P.tiles[t + 3] + lb});
        }
        std::copy(P.rec.begin(), P.rec.end(), hm.hal_rec.begin() + (size_t)2 * hm.state_base[m]);
        hm.hal_list.insert(hm.hal_list.end(), P.list.begin(), P.list.end());
        P = Part();
    }
    hm.hal_tile_base[M] = (int32_t)(hm.hal_tile.size() / 4);
    // the sweep trusts this layout for its LDS and HBM addresses: check it
    // (every state in exactly one tile of its model, halo places in range and
    // naming the record's successors, own states first)
    std::vector<uint8_t> seen((size_t)S, 0);
    for (int m = 0; m < M; ++m)
        for (int32_t t = hm.hal_tile_base[m]; t < hm.hal_tile_base[m + 1]; ++t) {
            const int32_t* T = &hm.hal_tile[(size_t)t * 4];
            const int32_t n = T[2] & 0xffff, H = T[2] >> 16, rb = T[1], hb = T[3];
            MORAP_CHECK(T[0] == m && n >= 1 && n <= HALO_TILE && H >= n && H <= HALO_MAX &&
                            rb >= hm.state_base[m] && rb + n <= hm.state_base[m + 1] && hb >= 0 &&
                            (size_t)hb + H <= hm.hal_list.size(),
                        MORAP_E_INVALID, "halo tiles: a tile out of its bounds");
            for (int32_t h = 0; h < H; ++h) {
                const int32_t g = hm.hal_list[(size_t)hb + h];
                MORAP_CHECK(g >= hm.state_base[m] && g < hm.state_base[m + 1], MORAP_E_INVALID,
                            "halo tiles: a row outside its model");
            }
            for (int32_t p = 0; p < n; ++p) {
                const int32_t g = hm.hal_list[(size_t)hb + p];
                MORAP_CHECK(!seen[g], MORAP_E_INVALID, "halo tiles: a state in two tiles");
                seen[g] = 1;
                const uint32_t w0 = hm.hal_rec[2 * (size_t)(rb + p)], w1 = hm.hal_rec[2 * (size_t)(rb + p) + 1];
                const uint32_t loc[NS] = {w0 & 255u, (w0 >> 8) & 255u, (w0 >> 16) & 255u, w0 >> 24, w1 & 255u};
                for (int d = 0; d < NS; ++d) {
                    const int32_t r = recs[(size_t)g * 8 + d];
                    const bool ok = r == S ? loc[d] == (uint32_t)HALO_MAX
                                           : (loc[d] < (uint32_t)H && hm.hal_list[(size_t)hb + loc[d]] == r);
                    MORAP_CHECK(ok, MORAP_E_INVALID, "halo tiles: a record slot names the wrong row");
                }
                MORAP_CHECK((w1 >> 13) == (uint32_t)recs[(size_t)g * 8 + 5] &&
                                ((w1 >> 8) & 31u) == ((uint32_t)recs[(size_t)g * 8 + 6] & 31u),
                            MORAP_E_INVALID, "halo tiles: a record's block or accepting slots differ");
            }
        }
    for (int32_t g = 0; g < S; ++g) MORAP_CHECK(seen[g], MORAP_E_INVALID, "halo tiles: a state in no tile");
}

// Neighbourhood-block form of built products (see the sweep over it): needs
// at most 5 actions per agent and at most 5 distinct successors per agent
// state, the state itself included; otherwise the form is not built and the
// CSR sweeps serve alone.
static void build_blocks(morap_ctx* c, const morap_agent* agents, int nI, const morap_dfa* tasks, int nJ,
                         const int32_t* const* letters) {
    HostModels& hm = c->hm;
    hm.blk_rec.clear();
    hm.blk_agent.clear();
    constexpr int NS = 5;
    std::vector<int64_t> abase(nI + 1, 0);
    for (int i = 0; i < nI; ++i) {
        if (agents[i].n_actions > NS) return;
        abase[i + 1] = abase[i] + agents[i].n_states;
    }
    if (abase[nI] >= (int64_t)1 << 30) return;
    // agent slots (slot 0 = the state itself) and blocks
    std::vector<int32_t> slot((size_t)abase[nI] * NS, -1);
    std::vector<uint8_t> amask((size_t)abase[nI], 0);
    std::vector<double> blk((size_t)abase[nI] * 32, 0.0);
    for (int i = 0; i < nI; ++i) {
        const morap_agent& a = agents[i];
        for (int s = 0; s < a.n_states; ++s) {
            const int64_t ab = abase[i] + s;
            // slots: 0 = the state itself, 1 + a = the most likely successor
            // of action a < 4 (on a grid: the cell the move aims at, so a
            // move's slips land in the slots of the perpendicular moves and
            // all blocks share one sparsity pattern), then any other successor
            int32_t* sl = &slot[(size_t)ab * NS];
            sl[0] = s;
            auto find = [&](int32_t v) {
                for (int d = 0; d < NS; ++d)
                    if (sl[d] == v) return d;
                return -1;
            };
            for (int act = 0; act + 1 < NS && act < a.n_actions; ++act) {
                const int64_t r = (int64_t)s * a.n_actions + act;
                int32_t best = -1;
                double bp = -1.0;
                for (int32_t e = a.sa_ptr[r]; e < a.sa_ptr[r + 1]; ++e)
                    if (a.prob[e] > bp) {
                        bp = a.prob[e];
                        best = a.succ[e];
                    }
                if (best >= 0 && find(best) < 0) sl[1 + act] = best;
            }
            double* B = &blk[(size_t)ab * 32];
            for (int act = 0; act < a.n_actions; ++act) {
                const int64_t r = (int64_t)s * a.n_actions + act;
                if (a.sa_ptr[r + 1] == a.sa_ptr[r]) continue;
                amask[ab] |= (uint8_t)(1u << act);
                B[25 + act] = -a.cost[r];
                for (int32_t e = a.sa_ptr[r]; e < a.sa_ptr[r + 1]; ++e) {
                    int d = find(a.succ[e]);
                    if (d < 0) {
                        d = find(-1);
                        if (d < 0) return;   // too many successors: no block form
                        sl[d] = a.succ[e];
                    }
                    B[act * NS + d] += a.prob[e];
                }
            }
            // a disabled action repeats the first enabled one: the maximum
            // over actions is unchanged and the sweep needs no branch on it
            int first = 0;
            while (!((amask[ab] >> first) & 1)) ++first;
            for (int act = 0; act < NS; ++act) {
                if ((amask[ab] >> act) & 1) continue;
                for (int d = 0; d < NS; ++d) B[act * NS + d] = B[first * NS + d];
                B[25 + act] = B[25 + first];
            }
        }
    }
    // identical blocks (same probabilities and costs) are stored once: grid
    // agents have a few dozen distinct ones, which then stay cache-resident
    std::vector<int32_t> uniq((size_t)abase[nI]);
    std::vector<double> ublk;
    {
        std::unordered_map<std::string, int32_t> seen;
        for (int64_t ab = 0; ab < abase[nI]; ++ab) {
            std::string key(reinterpret_cast<const char*>(&blk[(size_t)ab * 32]), 32 * sizeof(double));
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(std::move(key), (int32_t)(ublk.size() / 32)).first;
                ublk.insert(ublk.end(), blk.begin() + ab * 32, blk.begin() + (ab + 1) * 32);
            }
            uniq[(size_t)ab] = it->second;
        }
    }
    // per product state records
    const int M = hm.M;
    const int32_t S = (int32_t)hm.S();
    std::vector<int32_t> recs((size_t)S * 8, 0);
    std::atomic<int> next{0};
    auto worker = [&] {
        std::vector<int32_t> map;
        std::vector<uint8_t> done;
        for (int m; (m = next++) < M;) {
            const int i = m / nJ, j = m % nJ;
            const morap_agent& a = agents[i];
            const morap_dfa& t = tasks[j];
            const int32_t* L = letters[m];
            const int32_t s0 = hm.state_base[m], s1 = hm.state_base[m + 1];
            if (s1 == s0) continue;
            done = done_locations(t);
            map.assign((size_t)a.n_states * t.n_locs, -1);
            for (int32_t g = s0; g < s1; ++g)
                map[(size_t)hm.states_sq[2 * (size_t)g + 1] * a.n_states + hm.states_sq[2 * (size_t)g]] = g;
            for (int32_t g = s0; g < s1; ++g) {
                const int s = hm.states_sq[2 * (size_t)g], q = hm.states_sq[2 * (size_t)g + 1];
                const int64_t ab = abase[i] + s;
                int32_t* r = &recs[(size_t)g * 8];
                int32_t acc = 0;
                for (int d = 0; d < NS; ++d) {
                    const int32_t s2 = slot[(size_t)ab * NS + d];
                    r[d] = S;
                    if (s2 < 0) continue;
                    const int q2 = t.delta[(int64_t)q * t.n_letters + L[s2]];
                    if (done[q2]) {
                        if (t.accepting[q2]) acc |= 1 << d;
                    } else {
                        r[d] = map[(size_t)q2 * a.n_states + s2];
                    }
                }
                r[5] = uniq[(size_t)ab];
                r[6] = acc | ((int32_t)amask[ab] << 8);
                r[7] = g;
            }
        }
    };
    const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k) th.emplace_back(worker);
    for (auto& k : th) k.join();
    for (size_t g = 0; g < (size_t)S; ++g)
        for (int d = 0; d < NS; ++d)
            MORAP_CHECK(recs[g * 8 + d] >= 0 && recs[g * 8 + d] <= S, MORAP_E_INVALID,
                        "neighbourhood block: a successor that is not a live state of the model");
    // union of the nonzero (action, slot) entries over all blocks
    uint32_t pat = 0;
    for (size_t b = 0; b < ublk.size() / 32; ++b)
        for (int e = 0; e < NS * NS; ++e)
            if (ublk[b * 32 + e] != 0.0) pat |= 1u << e;
    hm.blk_pattern = pat;
    build_halo(hm, abase, slot, nI, nJ, recs, (int64_t)(ublk.size() / 32));
    hm.blk_rec = std::move(recs);
    hm.blk_agent = std::move(ublk);
}

void product_host(const morap_agent* a, const morap_dfa* t, const int32_t* letters, int32_t* sizes,
                  int32_t* state_row, int32_t* row_ptr, int32_t* col, double* prob, double* rew, uint8_t* to_done,
                  int32_t* states) {
    MORAP_CHECK(a && t && letters && sizes, MORAP_E_INVALID, "bad arguments");
    validate_agent(*a, 0);
    validate_dfa(*t, 0);
    for (int s = 0; s < a->n_states; ++s)
        MORAP_CHECK(letters[s] >= 0 && letters[s] < t->n_letters, MORAP_E_INVALID, "letter out of range");
    const Built b = build_one(*a, *t, letters);
    const size_t lim = 0x7fffffff;
    MORAP_CHECK(b.state_row.size() <= lim && b.row_ptr.size() <= lim && b.col.size() < lim, MORAP_E_UNSUPPORTED,
                "more than 2^31-1 states, rows or entries");
    const int32_t S = (int32_t)b.state_row.size() - 1, R = (int32_t)b.row_ptr.size() - 1, N = (int32_t)b.col.size();
    sizes[0] = S;
    sizes[1] = R;
    sizes[2] = N;
    sizes[3] = b.init;
    if (state_row) std::copy(b.state_row.begin(), b.state_row.end(), state_row);
    if (row_ptr) std::copy(b.row_ptr.begin(), b.row_ptr.end(), row_ptr);
    if (col) std::copy(b.col.begin(), b.col.end(), col);
    if (prob) std::copy(b.prob.begin(), b.prob.end(), prob);
    if (rew) std::copy(b.rew.begin(), b.rew.end(), rew);
    if (to_done) std::copy(b.to_done.begin(), b.to_done.end(), to_done);
    if (states) std::copy(b.states_sq.begin(), b.states_sq.end(), states);
}

void build_products(morap_ctx* c, const morap_agent* agents, int nI, const morap_dfa* tasks, int nJ,
                    const int32_t* const* letters) {
    MORAP_CHECK(agents && tasks && letters && nI > 0 && nJ > 0, MORAP_E_INVALID, "bad arguments");
    for (int i = 0; i < nI; ++i) validate_agent(agents[i], i);
    for (int j = 0; j < nJ; ++j) validate_dfa(tasks[j], j);
    for (int i = 0; i < nI; ++i)
        for (int j = 0; j < nJ; ++j) {
            const int32_t* l = letters[(size_t)i * nJ + j];
            MORAP_CHECK(l != nullptr, MORAP_E_INVALID, "NULL letters");
            for (int s = 0; s < agents[i].n_states; ++s)
                MORAP_CHECK(l[s] >= 0 && l[s] < tasks[j].n_letters, MORAP_E_INVALID, "letter out of range");
        }
    const int M = nI * nJ;
    std::vector<Built> parts(M);
    std::atomic<int> next{0};
    std::string err;
    std::atomic<bool> bad{false};
    auto worker = [&] {
        for (int m; (m = next++) < M;) {
            try {
                parts[m] = build_one(agents[m / nJ], tasks[m % nJ], letters[m]);
            } catch (...) {
                bad = true;
            }
        }
    };
    const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
    MORAP_CHECK(!bad, MORAP_E_OOM, "product construction failed (host memory)");
    concat(c, parts, nI, nJ);
    build_blocks(c, agents, nI, tasks, nJ, letters);
    upload_models(c);
}

void load_models(morap_ctx* c, const morap_model* models, int n, int nI, int nJ) {
    MORAP_CHECK(models && nI > 0 && nJ > 0 && n == nI * nJ, MORAP_E_INVALID, "need n_models = n_agents * n_tasks");
    std::vector<Built> parts(n);
    for (int m = 0; m < n; ++m) {
        const morap_model& md = models[m];
        const std::string who = "model " + std::to_string(m) + ": ";
        MORAP_CHECK(md.agent == m / nJ && md.task == m % nJ, MORAP_E_INVALID, who + "agent/task do not match m");
        MORAP_CHECK(md.n_states >= 0 && md.n_rows >= 0 && md.nnz >= 0, MORAP_E_INVALID, who + "negative size");
        MORAP_CHECK(md.init >= -1 && md.init < md.n_states, MORAP_E_INVALID, who + "init out of range");
        MORAP_CHECK(md.n_states == 0 || (md.state_row && md.row_ptr && md.rew && md.to_done), MORAP_E_INVALID,
                    who + "NULL arrays");
        Built& b = parts[m];
        b.init = md.init;
        if (md.n_states == 0) continue;
        MORAP_CHECK(md.state_row[0] == 0 && md.state_row[md.n_states] == md.n_rows, MORAP_E_INVALID,
                    who + "state_row must run from 0 to n_rows");
        MORAP_CHECK(md.row_ptr[0] == 0 && md.row_ptr[md.n_rows] == md.nnz, MORAP_E_INVALID,
                    who + "row_ptr must run from 0 to nnz");
        b.state_row.assign(md.state_row, md.state_row + md.n_states + 1);
        b.row_ptr.assign(md.row_ptr, md.row_ptr + md.n_rows + 1);
        for (int s = 0; s < md.n_states; ++s)
            MORAP_CHECK(md.state_row[s + 1] > md.state_row[s], MORAP_E_INVALID, who + "a state without rows");
        for (int r = 0; r < md.n_rows; ++r) {
            MORAP_CHECK(md.row_ptr[r + 1] >= md.row_ptr[r], MORAP_E_INVALID, who + "row_ptr not monotone");
            double sum = 0;
            for (int e = md.row_ptr[r]; e < md.row_ptr[r + 1]; ++e) {
                MORAP_CHECK(md.col[e] >= 0 && md.col[e] < md.n_states, MORAP_E_INVALID, who + "col out of range");
                MORAP_CHECK(std::isfinite(md.prob[e]) && md.prob[e] >= 0, MORAP_E_INVALID, who + "bad probability");
                sum += md.prob[e];
            }
            MORAP_CHECK(sum <= 1.0 + 1e-6, MORAP_E_INVALID, who + "a row sums above 1");
            MORAP_CHECK(std::isfinite(md.rew[2 * r]) && std::isfinite(md.rew[2 * r + 1]), MORAP_E_INVALID,
                        who + "non-finite reward");
        }
        b.col.assign(md.col, md.col + md.nnz);
        b.prob.assign(md.prob, md.prob + md.nnz);
        b.rew.assign(md.rew, md.rew + 2 * (size_t)md.n_rows);
        b.to_done.assign(md.to_done, md.to_done + md.n_rows);
        b.states_sq.assign((size_t)2 * md.n_states, 0);
    }
    concat(c, parts, nI, nJ);
    upload_models(c);
}

template <class T>
static void upload(morap::DevBuf& d, const std::vector<T>& h, hipStream_t s) {
    d.ensure(h.size() * sizeof(T) + 16);
    if (!h.empty()) MORAP_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Order of the neighbourhood-block records inside every tile (a record
// carries its state in [7]).  With the grid slot order (slot 1 / 2 = the
// state a north / south move aims at) a tile is walked column by column:
// vertical neighbours follow each other and the tiles processed side by side
// reach the same columns at about the same time, so every successor row is
// reused from cache soon after it is first fetched.  Otherwise state order.
static void order_records(morap_ctx* c) {
    HostModels& hm = c->hm;
    const int64_t S = hm.S();
    // back to state order (idempotent)
    {
        std::vector<int32_t> nat(hm.blk_rec.size());
        for (int64_t p = 0; p < S; ++p) {
            const int32_t g = hm.blk_rec[(size_t)p * 8 + 7];
            std::copy(&hm.blk_rec[(size_t)p * 8], &hm.blk_rec[(size_t)p * 8 + 8], &nat[(size_t)g * 8]);
        }
        hm.blk_rec.swap(nat);
    }
    constexpr uint32_t kGridPattern = (1u << 0) | (1u << 1) | (1u << 3) | (1u << 4) | (1u << 5) | (1u << 7) |
                                      (1u << 8) | (1u << 9) | (1u << 10) | (1u << 11) | (1u << 12) |
                                      (1u << 13) | (1u << 15) | (1u << 16) | (1u << 17) | (1u << 19) | (1u << 20);
    if ((hm.blk_pattern & ~kGridPattern) != 0) return;
    std::vector<int32_t> out(hm.blk_rec.size());
    std::vector<int> order, up, down;
    std::vector<uint8_t> seen;
    for (const Tile& t : c->tiles) {
        const int b = t.s_begin, n = t.s_end - t.s_begin;
        auto local = [&](int32_t g) { return (g >= b && g < b + n) ? g - b : -1; };
        up.assign(n, -1);
        down.assign(n, -1);
        seen.assign(n, 0);
        order.clear();
        for (int i = 0; i < n; ++i) {
            up[i] = local(hm.blk_rec[(size_t)(b + i) * 8 + 1]);
            down[i] = local(hm.blk_rec[(size_t)(b + i) * 8 + 2]);
        }
        for (int i = 0; i < n; ++i) {
            if (seen[i]) continue;
            int j = i;
            for (int steps = 0; steps < n && up[j] >= 0 && !seen[up[j]] && up[j] != i; ++steps) j = up[j];
            for (int from : {j, i})   // from i too when the column above does not lead back to it
                for (int k = from; k >= 0 && !seen[k]; k = down[k]) {
                    seen[k] = 1;
                    order.push_back(k);
                }
        }
        MORAP_CHECK((int)order.size() == n, MORAP_E_INVALID, "record order is not a permutation");
        for (int p = 0; p < n; ++p)
            std::copy(&hm.blk_rec[(size_t)(b + order[p]) * 8], &hm.blk_rec[(size_t)(b + order[p]) * 8 + 8],
                      &out[(size_t)(b + p) * 8]);
    }
    hm.blk_rec.swap(out);
}

void upload_models(morap_ctx* c) {
    const HostModels& hm = c->hm;
    hipStream_t s = c->stream;
    c->loaded = false;
    c->solved = false;
    c->evaluated = false;
    c->team = false;
    c->tuned.clear();
    c->resident.clear();
    // captured sweep graphs bake in the model buffers, the zero row and the
    // block pattern: none of them may replay after a new upload
    ++c->load_gen;
    c->S = hm.S();
    c->R = hm.R();
    c->N = hm.N();
    upload(c->d_state_row, hm.state_row, s);
    upload(c->d_row_ptr, hm.row_ptr, s);
    upload(c->d_col, hm.col, s);
    upload(c->d_prob64, hm.prob, s);
    upload(c->d_rew64, hm.rew, s);
    upload(c->d_to_done, hm.to_done, s);
    upload(c->d_state_base, hm.state_base, s);
    {
        std::vector<int32_t> sm((size_t)c->S);
        for (int m = 0; m < hm.M; ++m)
            std::fill(sm.begin() + hm.state_base[m], sm.begin() + hm.state_base[m + 1], m);
        upload(c->d_state_model, sm, s);
        MORAP_HIP(hipStreamSynchronize(s));   // sm goes out of scope
    }
    upload(c->d_init, hm.init, s);
    // FP32 copies for FP32 sweeps
    c->d_prob32.ensure((size_t)c->N * 4 + 16);
    c->d_rew32.ensure((size_t)c->R * 8 + 16);
    k::to_f32(s, c->d_prob64.as<double>(), c->d_prob32.as<float>(), c->N);
    k::to_f32(s, c->d_rew64.as<double>(), c->d_rew32.as<float>(), 2 * c->R);
    // per-model sizes for the traffic and backup counters
    std::vector<int32_t> rows(hm.M), states(hm.M);
    std::vector<int64_t> b32(hm.M), b64(hm.M);
    for (int m = 0; m < hm.M; ++m) {
        const int32_t s0 = hm.state_base[m], s1 = hm.state_base[m + 1];
        states[m] = s1 - s0;
        rows[m] = hm.state_row[s1] - hm.state_row[s0];
        const int64_t nnz = hm.row_ptr[hm.state_row[s1]] - hm.row_ptr[hm.state_row[s0]];
        // state_row + row_ptr + col (int32) + prob + two rewards per row
        b32[m] = 4 * (int64_t)states[m] + 4 * (int64_t)rows[m] + 4 * nnz + 4 * nnz + 8 * (int64_t)rows[m];
        b64[m] = 4 * (int64_t)states[m] + 4 * (int64_t)rows[m] + 4 * nnz + 8 * nnz + 16 * (int64_t)rows[m];
    }
    upload(c->d_rows_per_model, rows, s);
    upload(c->d_states_per_model, states, s);
    upload(c->d_csr_bytes32, b32, s);
    upload(c->d_csr_bytes64, b64, s);
    // tiles: consecutive states of one model within the LDS limits
    c->tiles.clear();
    c->tile_base.assign(hm.M + 1, 0);
    const int TS = k::sweep_tile_states(Variant{0, 1, 1, 64}), TR = k::sweep_lds_rows(), TN = k::sweep_lds_nnz();
    for (int m = 0; m < hm.M; ++m) {
        c->tile_base[m] = (int32_t)c->tiles.size();
        int32_t s = hm.state_base[m];
        const int32_t s_end = hm.state_base[m + 1];
        while (s < s_end) {
            int32_t e = s;
            while (e < s_end && e - s < TS) {
                const int32_t rows_t = hm.state_row[e + 1] - hm.state_row[s];
                const int32_t nnz_t = hm.row_ptr[hm.state_row[e + 1]] - hm.row_ptr[hm.state_row[s]];
                if (rows_t > TR || nnz_t > TN) break;
                ++e;
            }
            MORAP_CHECK(e > s, MORAP_E_UNSUPPORTED, "a state's rows or entries exceed the tile staging limits");
            c->tiles.push_back(Tile{m, s, e, 0});
            s = e;
        }
    }
    c->tile_base[hm.M] = (int32_t)c->tiles.size();
    upload(c->d_tiles, c->tiles, s);
    upload(c->d_tile_base, c->tile_base, s);
    c->has_blocks = !hm.blk_rec.empty();
    c->has_halo = c->has_blocks && !hm.hal_tile.empty();
    c->n_htiles = (int64_t)hm.hal_tile.size() / 4;
    if (c->has_halo) {
        upload(c->d_htiles, hm.hal_tile, s);
        upload(c->d_htile_base, hm.hal_tile_base, s);
        upload(c->d_hrec, hm.hal_rec, s);
        upload(c->d_hlist, hm.hal_list, s);
    }
    if (c->has_blocks) {
        order_records(c);
        upload(c->d_blk_rec, hm.blk_rec, s);
        upload(c->d_blk64, hm.blk_agent, s);
        c->d_blk32.ensure(hm.blk_agent.size() * 4 + 16);
        k::to_f32(s, c->d_blk64.as<double>(), c->d_blk32.as<float>(), (int64_t)hm.blk_agent.size());
    }
    MORAP_HIP(hipStreamSynchronize(s));
    c->loaded = true;
}

// A team model's optimum from value iteration started at 0 can be improper:
// where an agent's steps weigh nothing it may take a task and never finish
// it, so the agents after it never start theirs (and spend nothing).  The
// optimum over proper policies -- the assignment optimum of Lemma
// lem:ct-mdp-prop -- is the least fixed point of the backup, and value
// iteration reaches it from any start below it.  The start used: the values
// of one fixed proper policy pi, per objective, E[s][o] (a solve starts each
// column at sum_o w[o] E[s][o]).  pi is the attractor policy of all rows
// (ranks are distances to done; each state takes the row moving the most
// mass into done or lower ranks), E its Jacobi evaluation on the device.
static void team_proper_start(morap_ctx* c, int d) {
    const HostModels& hm = c->hm;
    const int64_t S = hm.S();
    // predecessors of every state (over all rows)
    std::vector<int64_t> pstart(S + 1, 0);
    for (int64_t s = 0; s < S; ++s)
        for (int32_t r = hm.state_row[s]; r < hm.state_row[s + 1]; ++r)
            for (int32_t e = hm.row_ptr[r]; e < hm.row_ptr[r + 1]; ++e) ++pstart[hm.col[e] + 1];
    for (int64_t s = 0; s < S; ++s) pstart[s + 1] += pstart[s];
    std::vector<int32_t> pred(pstart[S]);
    {
        std::vector<int64_t> fill(pstart.begin(), pstart.end() - 1);
        for (int64_t s = 0; s < S; ++s)
            for (int32_t r = hm.state_row[s]; r < hm.state_row[s + 1]; ++r)
                for (int32_t e = hm.row_ptr[r]; e < hm.row_ptr[r + 1]; ++e) pred[fill[hm.col[e]]++] = (int32_t)s;
    }
    // BFS ranks from done
    std::vector<int32_t> rank(S, -1), queue;
    queue.reserve(S);
    for (int64_t s = 0; s < S; ++s)
        for (int32_t r = hm.state_row[s]; r < hm.state_row[s + 1]; ++r)
            if (hm.to_done[r] && rank[s] < 0) {
                rank[s] = 1;
                queue.push_back((int32_t)s);
            }
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t t = queue[h];
        for (int64_t p = pstart[t]; p < pstart[t + 1]; ++p)
            if (rank[pred[p]] < 0) {
                rank[pred[p]] = rank[t] + 1;
                queue.push_back(pred[p]);
            }
    }
    std::vector<int32_t> pi(S);
    for (int64_t s = 0; s < S; ++s) {
        MORAP_CHECK(rank[s] >= 0, MORAP_E_INVALID, "team model: a state cannot reach done");
        int best = -1;
        double best_m = -1.0;
        for (int32_t r = hm.state_row[s]; r < hm.state_row[s + 1]; ++r) {
            double m = 0.0, live = 0.0;
            bool hit = hm.to_done[r] != 0;
            for (int32_t e = hm.row_ptr[r]; e < hm.row_ptr[r + 1]; ++e) {
                live += hm.prob[e];
                if (rank[hm.col[e]] < rank[s]) {
                    hit = true;
                    m += hm.prob[e];
                }
            }
            if (hm.to_done[r]) m += 1.0 - live;
            if (hit && m > best_m + 1e-12) {
                best_m = m;
                best = r;
            }
        }
        pi[s] = best;
    }
    upload(c->d_team_pi, pi, c->stream);
    hipStream_t st = c->stream;
    morap::DevBuf E1, res;
    c->d_team_E.ensure((size_t)S * d * 8 + 8);
    E1.ensure((size_t)S * d * 8 + 8);
    res.ensure(8);
    double* e0 = c->d_team_E.as<double>();
    double* e1 = E1.as<double>();
    k::fill_f64(st, e0, 0.0, S * d);
    int64_t sweeps = 0;
    while (true) {
        unsigned long long r = 0;
        for (int i = 0; i < 64; ++i) {
            if (i == 63) MORAP_HIP(hipMemsetAsync(res.p, 0, 8, st));
            k::team_eval_sweep(st, S, d, c->d_team_pi.as<int32_t>(), c->d_row_ptr.as<int32_t>(),
                               c->d_col.as<int32_t>(), c->d_prob64.as<double>(), c->d_rew64.as<double>(),
                               c->d_obj.as<int32_t>(), (i & 1) ? e1 : e0, (i & 1) ? e0 : e1,
                               i == 63 ? res.as<unsigned long long>() : nullptr);
        }
        sweeps += 64;
        MORAP_HIP(hipMemcpyAsync(&r, res.p, 8, hipMemcpyDeviceToHost, st));
        MORAP_HIP(hipStreamSynchronize(st));
        double change;
        std::memcpy(&change, &r, 8);
        if (change <= 1e-12) break;
        MORAP_CHECK(sweeps < 10000000, MORAP_E_NOT_CONVERGED, "team model: evaluation of the start policy");
    }
}

// A team MDP (Def. teamMDP) with its d objectives: one caller-built model
// plus the objective of each of a row's two rewards.
void load_team_model(morap_ctx* c, int nA, int nT, const morap_model* model, const int32_t* obj) {
    MORAP_CHECK(model && obj && nA >= 1 && nT >= 1 && nA + nT <= 4096, MORAP_E_INVALID,
                "bad team model arguments");
    MORAP_CHECK(model->agent == 0 && model->task == 0, MORAP_E_INVALID, "a team model has agent = task = 0");
    MORAP_CHECK(model->n_rows >= 0, MORAP_E_INVALID, "negative size");
    const int d = nA + nT;
    for (int64_t r = 0; r < 2 * (int64_t)model->n_rows; ++r)
        MORAP_CHECK(obj[r] >= 0 && obj[r] < d, MORAP_E_INVALID, "objective index out of range");
    load_models(c, model, 1, 1, 1);
    c->loaded = false;
    std::vector<int32_t> o(obj, obj + 2 * (size_t)model->n_rows);
    upload(c->d_obj, o, c->stream);
    team_proper_start(c, d);
    c->team = true;
    c->team_nI = nA;
    c->team_nJ = nT;
    c->loaded = true;
}

}  // namespace morap
