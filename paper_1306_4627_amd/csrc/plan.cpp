// plan.cpp -- packing of LCS pairs into wave-sized work items (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>

namespace lcs {

static inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Words-per-lane chosen automatically from the number of 64-bit words of a
// pair: short columns keep all lanes busy with one word each; long columns
// amortise the per-step overhead over more words per lane.
//
// Limits from the kernel: the fill keeps the match masks of its waves in
// LDS, (sigma+1) * wpl * 512 bytes per wave, with four, two or one waves per
// work-group, so (sigma+1) * wpl * 512 <= 160 KiB.  The stream element is
// the code already shifted to its LDS row, code << log2(wpl*512), when that
// fits 16 bits (sigma * wpl <= 127); otherwise ("raw" stream, wpl 1 or 2)
// it is the plain code and the fill shifts it.  Where possible the batch
// keeps (sigma+1) * wpl <= 40, so that a second work-group fits a compute
// unit.
bool raw_stream(int sigma, int wpl) { return sigma * wpl > 127; }

int fill_waves(int sigma, int wpl) {
    // LDS of one wave: its match masks ([symbol + sentinel][word][lane]) and
    // the threshold pass's 128 words; the work-group size (4, 2 or 1 waves;
    // the waves are independent) that keeps the most waves resident on a
    // 160 KiB CU wins, up to 16 (four per SIMD, what the fill's registers
    // allow), larger groups on ties
    const size_t per_wave = (size_t)(sigma + 1) * wpl * 512 + 512;
    const size_t lds = 160 * 1024;
    int best = 0, best_res = 0;
    for (int w = 4; w >= 1; w >>= 1) {
        if ((size_t)w * per_wave > lds) continue;
        const int res = std::min<int>((int)(lds / ((size_t)w * per_wave)) * w, 16);
        if (res > best_res) {
            best = w;
            best_res = res;
        }
    }
    return best;
}

bool wpl_fits(int sigma, int wpl) {
    if (sigma < 1 || sigma > 256) return false;
    if (wpl != 1 && wpl != 2 && wpl != 4 && wpl != 8) return false;
    if (raw_stream(sigma, wpl) && wpl > 2) return false;
    return fill_waves(sigma, wpl) > 0;
}

int max_wpl(int sigma) {
    for (int w = 8; w >= 1; w >>= 1)
        if ((sigma + 1) * w <= 40 && wpl_fits(sigma, w)) return w;
    return wpl_fits(sigma, 1) ? 1 : 0;
}

// One words-per-lane for the whole batch (one fill launch).  When every
// lane of the batch at one word per lane fits the GPU's resident wave slots
// at once (compute units x 16 waves x 64 lanes), the fill is bound by the latency
// of a step, which grows with the words in a lane's carry chain: one word
// (a single 262144-row pair: 12.0 ms against 15.0 at two words).
// Otherwise two words per lane once most of the cells belong to pairs
// longer than 16 words (the per-step overhead is then spread over 128
// rows), one word otherwise (short columns keep more lanes busy).
static int auto_batch_wpl(const std::vector<PairShape> &pairs, int sigma, int cus) {
    const uint64_t resident_lanes = (uint64_t)std::max(cus, 1) * 16 * kLanes;
    double big = 0, all = 0;
    uint64_t lanes1 = 0;
    for (const PairShape &p : pairs) {
        const double c = (double)p.m * (double)p.n;
        all += c;
        if ((p.m + 63) / 64 > 16) big += c;
        if (p.n) lanes1 += (p.m + 63) / 64;
    }
    int w = (all > 0 && big >= 0.5 * all && lanes1 > resident_lanes) ? 2 : 1;
    int mw = max_wpl(sigma);
    return w < mw ? w : mw;
}

// History of one item in the round buffer, uint64 words: V checkpoints,
// then the carry-in words (two per uint64 word).
static uint64_t item_ck_words(const ClassPlan &C, size_t it, int ckpt) {
    return ceil_div(C.it_T[it], (uint64_t)ckpt) * (uint64_t)C.wpl * kLanes;
}
static uint64_t item_cb_words(const ClassPlan &C, size_t it) {
    return (C.it_T[it] / kCbitsPer) * kLanes;
}
static uint64_t item_round_words(const ClassPlan &C, size_t it, int ckpt) {
    return item_ck_words(C, it, ckpt) + ceil_div(item_cb_words(C, it), 2);
}

// Rounds of the traceback (PlanConfig::round_bytes): items are given to
// rounds chain by chain from the top, as many consecutive items of a chain
// per round as fit, chains with the most items left first; every round's
// histories fit round_bytes.  Then each traceback entry's strips are grouped
// by the round of the items that hold them (strips never straddle items).
static std::string plan_rounds(const std::vector<PairShape> &pairs, const PlanConfig &cfg, ClassPlan &C) {
    const size_t nit = C.it_T.size();
    const uint64_t cap_words = cfg.round_bytes / 8;
    for (size_t it = 0; it < nit; ++it)
        if (item_round_words(C, it, cfg.ckpt) > cap_words) return "item history exceeds the round capacity";
    // chains: [bottom item, top item]
    std::vector<std::pair<uint32_t, uint32_t>> chains;
    for (size_t it = 0; it < nit; ++it) {
        if (C.it_prev[it] < 0) chains.push_back({(uint32_t)it, (uint32_t)it});
        else chains.back().second = (uint32_t)it;
    }
    std::vector<int64_t> next(chains.size());
    for (size_t c = 0; c < chains.size(); ++c) next[c] = chains[c].second;
    C.it_round.assign(nit, UINT32_MAX);
    C.it_rb.assign(nit, 0);
    C.it_rcb.assign(nit, 0);
    C.rd_item_off.assign(1, 0);
    C.rd_items.clear();
    std::vector<size_t> order(chains.size());
    std::iota(order.begin(), order.end(), 0);
    size_t left = nit;
    uint32_t r = 0;
    while (left) {
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            return next[a] - (int64_t)chains[a].first > next[b] - (int64_t)chains[b].first;
        });
        uint64_t used = 0;
        for (size_t c : order) {
            while (next[c] >= (int64_t)chains[c].first) {
                const size_t it = (size_t)next[c];
                const uint64_t w = item_round_words(C, it, cfg.ckpt);
                if (used + w > cap_words) break;
                C.it_round[it] = r;
                C.it_rb[it] = used;
                C.it_rcb[it] = 2 * (used + item_ck_words(C, it, cfg.ckpt));
                C.rd_items.push_back((uint32_t)it);
                used += w;
                --next[c];
                --left;
            }
        }
        if (used == 0) return "round scheduling made no progress";
        C.round_words = std::max(C.round_words, used);
        C.rd_item_off.push_back((uint32_t)C.rd_items.size());
        ++r;
    }
    C.n_rounds = r;
    // tickets per round
    std::vector<std::vector<uint32_t>> sp_t(r), sp_s(r), fx_t(r), fx_s(r), sl_t(r), sl_top(r), sl_lo(r);
    std::vector<std::vector<uint64_t>> sp_est(r);
    const uint64_t band = (uint64_t)kLanes * C.wpl;
    const uint64_t R = (uint64_t)C.strip_bands * band;
    for (size_t t = 0; t < C.tb_pair.size(); ++t) {
        const PairShape &ps = pairs[C.tb_pair[t]];
        const uint64_t nb = ceil_div(ps.m, band);
        const uint64_t S = ceil_div(nb, (uint64_t)C.strip_bands);
        auto round_of_band = [&](uint64_t b) {
            return C.it_round[C.tb_item[t] + (C.tb_lane0[t] + b) / kLanes];
        };
        uint64_t s = S;
        while (s-- > 0) {
            const uint64_t top = s;
            const uint32_t rr = round_of_band(top * C.strip_bands);
            for (uint64_t b = top * C.strip_bands; b < std::min(nb, (top + 1) * C.strip_bands); ++b)
                if (round_of_band(b) != rr) return "strip straddles two rounds";
            uint64_t lo = top;
            while (lo > 0 && round_of_band((lo - 1) * C.strip_bands) == rr) --lo;
            for (uint64_t q = top + 1; q-- > lo;) {
                sp_t[rr].push_back((uint32_t)t);
                sp_s[rr].push_back((uint32_t)q | ((q == top && top + 1 < S) ? kFromAbove : 0u));
                const uint64_t lo_row = q * R;
                const uint64_t rows = std::min<uint64_t>(R, ps.m - lo_row);
                sp_est[rr].push_back(rows + (ps.m ? (uint64_t)((double)ps.n * (double)rows / (double)ps.m) : 0));
                if (q < top) {
                    fx_t[rr].push_back((uint32_t)t);
                    fx_s[rr].push_back((uint32_t)q);
                }
            }
            if (top > lo) {
                sl_t[rr].push_back((uint32_t)t);
                sl_top[rr].push_back((uint32_t)top);
                sl_lo[rr].push_back((uint32_t)lo);
            }
            s = lo;
        }
    }
    C.rd_sp_off.assign(1, 0);
    C.rd_fx_off.assign(1, 0);
    C.rd_sl_off.assign(1, 0);
    C.rd_sp_t.clear(); C.rd_sp_s.clear(); C.rd_fx_t.clear(); C.rd_fx_s.clear();
    C.rd_sl_t.clear(); C.rd_sl_top.clear(); C.rd_sl_lo.clear();
    for (uint32_t q = 0; q < r; ++q) {
        // speculative strips longest walk first within the round
        std::vector<size_t> o(sp_t[q].size());
        std::iota(o.begin(), o.end(), 0);
        std::stable_sort(o.begin(), o.end(), [&](size_t x, size_t y) { return sp_est[q][x] > sp_est[q][y]; });
        for (size_t k : o) {
            C.rd_sp_t.push_back(sp_t[q][k]);
            C.rd_sp_s.push_back(sp_s[q][k]);
        }
        C.rd_fx_t.insert(C.rd_fx_t.end(), fx_t[q].begin(), fx_t[q].end());
        C.rd_fx_s.insert(C.rd_fx_s.end(), fx_s[q].begin(), fx_s[q].end());
        C.rd_sl_t.insert(C.rd_sl_t.end(), sl_t[q].begin(), sl_t[q].end());
        C.rd_sl_top.insert(C.rd_sl_top.end(), sl_top[q].begin(), sl_top[q].end());
        C.rd_sl_lo.insert(C.rd_sl_lo.end(), sl_lo[q].begin(), sl_lo[q].end());
        C.rd_sp_off.push_back((uint32_t)C.rd_sp_t.size());
        C.rd_fx_off.push_back((uint32_t)C.rd_fx_t.size());
        C.rd_sl_off.push_back((uint32_t)C.rd_sl_t.size());
    }
    return std::string();
}

std::string build_plan(const std::vector<PairShape> &pairs, const PlanConfig &cfg, Plan &out) {
    out = Plan();
    out.cfg = cfg;
    if (cfg.wpl != 0 && cfg.wpl != 1 && cfg.wpl != 2 && cfg.wpl != 4 && cfg.wpl != 8)
        return "words_per_lane must be 1, 2, 4 or 8";
    if (cfg.traceback && cfg.ckpt != 64 && cfg.ckpt != 128 && cfg.ckpt != 256)
        return "ckpt_interval must be 64, 128 or 256";
    if (cfg.round_bytes && (!cfg.traceback || cfg.plain || cfg.link_items > 1))
        return "traceback rounds need a packed traceback batch without linked items";
    const size_t np = pairs.size();
    out.pair_class.assign(np, UINT32_MAX);

    const int batch_wpl = cfg.wpl ? cfg.wpl : auto_batch_wpl(pairs, cfg.sigma, cfg.cus);
    // assign pairs to classes by words-per-lane
    int class_of_wpl[9];
    for (int &c : class_of_wpl) c = -1;
    std::vector<std::vector<uint32_t>> members;
    for (size_t k = 0; k < np; ++k) {
        const PairShape &p = pairs[k];
        out.cells += p.m * p.n;
        if (p.m == 0 || p.n == 0) continue;
        int wpl = batch_wpl;
        // a pair too long for the batch's width takes a wider one
        while (wpl < 8 && p.m > max_rows(wpl)) wpl *= 2;
        if (wpl == 0 || !wpl_fits(cfg.sigma, wpl)) return "alphabet too large for words_per_lane";
        if (p.m > max_rows(wpl)) return "sequence X longer than the supported row count";
        if (p.n > 0x7fffffffull) return "sequence Y too long";
        if (class_of_wpl[wpl] < 0) {
            class_of_wpl[wpl] = (int)out.classes.size();
            out.classes.emplace_back();
            out.classes.back().wpl = wpl;
            members.emplace_back();
        }
        out.pair_class[k] = (uint32_t)class_of_wpl[wpl];
        members[class_of_wpl[wpl]].push_back((uint32_t)k);
    }

    // Y stream: a leading all-sentinel region read by idle lanes; its length
    // is fixed once max_T is known, so regions are laid out afterwards.
    struct PendingSeg { uint32_t pair; uint32_t pre; uint32_t last_item; uint32_t cls; };
    std::vector<PendingSeg> pend;

    for (size_t ci = 0; ci < out.classes.size(); ++ci) {
        ClassPlan &C = out.classes[ci];
        const int wpl = C.wpl;
        std::vector<uint32_t> &mem = members[ci];
        std::stable_sort(mem.begin(), mem.end(), [&](uint32_t a, uint32_t b) {
            if (pairs[a].n != pairs[b].n) return pairs[a].n > pairs[b].n;
            return pairs[a].m > pairs[b].m;
        });
        int64_t cur_item = -1;
        int cur_lane = kLanes;
        // the run of items linked by carry hand-over that ends with cur_item:
        // its largest step need and its length in items
        uint64_t run_need = 0;
        int run_len = 0;
        // segments of each item, to set T afterwards
        std::vector<std::vector<uint32_t>> item_segs;   // indices into pend
        auto new_item = [&](int32_t prev) {
            C.it_T.push_back(0);
            C.it_prev.push_back(prev);
            C.it_feeds.push_back(0);
            C.it_depth.push_back(prev >= 0 ? C.it_depth[prev] + 1 : 0);
            for (int l = 0; l < kLanes; ++l) {
                C.ln_pair.push_back(-1);
                C.ln_word0.push_back(0);
                C.ln_skew.push_back(0);
                C.ln_ys.push_back(0);
            }
            item_segs.emplace_back();
            return (int64_t)C.it_T.size() - 1;
        };
        for (uint32_t k : mem) {
            const PairShape &p = pairs[k];
            const uint64_t W = ceil_div(p.m, 64);
            const uint64_t s = ceil_div(W, (uint64_t)wpl);
            const uint32_t seg_id = (uint32_t)pend.size();
            if (s <= (uint64_t)kLanes) {
                if (cur_item < 0 || cur_lane + (int)s > kLanes || (cfg.plain && cur_lane > 0)) {
                    cur_item = new_item(-1);
                    cur_lane = 0;
                    run_need = 0;
                    run_len = 1;
                }
                run_need = std::max<uint64_t>(run_need, p.n + s);
                for (uint64_t l = 0; l < s; ++l) {
                    size_t li = (size_t)cur_item * kLanes + cur_lane + l;
                    C.ln_pair[li] = (int32_t)k;
                    C.ln_word0[li] = (uint32_t)(l * wpl);
                    C.ln_skew[li] = (uint32_t)l;
                }
                C.tb_pair.push_back(k);
                C.tb_item.push_back((uint32_t)cur_item);
                C.tb_lane0.push_back((uint32_t)cur_lane);
                pend.push_back({k, (uint32_t)(s - 1), (uint32_t)cur_item, (uint32_t)ci});
                item_segs[cur_item].push_back(seg_id);
                cur_lane += (int)s;
            } else {
                // A chain: lane g of the pair (words g*wpl..) sits g lanes
                // above its first lane, crossing into the next item after lane
                // 63, with a skew of g plus kChunk - 1 per item boundary
                // crossed (lane 0 of the next item takes lane 63's carry of
                // the chunk before, through memory).  It starts in the free
                // lanes of the current item when its step need is close to
                // that of the items already linked to it and the linked run
                // stays within link_items; else in a new item.
                auto need_at = [&](uint64_t l0) {
                    const uint64_t g = s - 1, q = (g + l0) / kLanes;
                    return p.n + g + (uint64_t)(kChunk - 1) * q + 1;
                };
                uint64_t l0 = 0;
                if (!cfg.plain && cur_item >= 0 && cur_lane < kLanes) {
                    const uint64_t need = need_at((uint64_t)cur_lane);
                    const uint64_t extra = ceil_div(s - (uint64_t)(kLanes - cur_lane), kLanes);
                    if ((double)need >= (1.0 - kLinkSpread) * (double)run_need &&
                        (double)need <= (1.0 + kLinkSpread) * (double)run_need &&
                        (uint64_t)run_len + extra <= (uint64_t)std::max(cfg.link_items, 1))
                        l0 = (uint64_t)cur_lane;
                }
                int64_t it = cur_item;
                if (l0 == 0) {
                    it = new_item(-1);
                    run_need = 0;
                    run_len = 1;
                }
                const int64_t first = it;
                uint64_t lane = l0, q = 0;
                for (uint64_t g = 0; g < s; ++g, ++lane) {
                    if (lane == (uint64_t)kLanes) {
                        C.it_feeds[it] = 1;
                        it = new_item((int32_t)it);
                        ++run_len;
                        lane = 0;
                        ++q;
                    }
                    const size_t li = (size_t)it * kLanes + lane;
                    C.ln_pair[li] = (int32_t)k;
                    C.ln_word0[li] = (uint32_t)(g * wpl);
                    C.ln_skew[li] = (uint32_t)(g + (uint64_t)(kChunk - 1) * q);
                    if (g == 0 || lane == 0) item_segs[it].push_back(seg_id);
                }
                const uint32_t pre = (uint32_t)(need_at(l0) - p.n - 1);
                run_need = std::max<uint64_t>(run_need, p.n + pre + 1);
                C.tb_pair.push_back(k);
                C.tb_item.push_back((uint32_t)first);
                C.tb_lane0.push_back((uint32_t)l0);
                pend.push_back({k, pre, (uint32_t)it, (uint32_t)ci});
                cur_item = it;
                cur_lane = (int)lane;
                if (cfg.plain) cur_lane = kLanes;
            }
        }
        // steps per item: every segment in it must reach column n at its
        // largest skew; chains share one step count
        const size_t nit = C.it_T.size();
        std::vector<uint64_t> T(nit, 0);
        for (size_t it = 0; it < nit; ++it)
            for (uint32_t sid : item_segs[it]) {
                const PendingSeg &ps = pend[sid];
                T[it] = std::max<uint64_t>(T[it], pairs[ps.pair].n + ps.pre + 1);
            }
        // propagate the maximum along chains (backwards then forwards)
        for (size_t it = nit; it-- > 1;)
            if (C.it_prev[it] >= 0) T[it - 1] = std::max(T[it - 1], T[it]);
        for (size_t it = 1; it < nit; ++it)
            if (C.it_prev[it] >= 0) T[it] = std::max(T[it], T[it - 1]);
        for (size_t it = 0; it < nit; ++it) {
            uint64_t t = ceil_div(std::max<uint64_t>(T[it], 1), kChunk) * kChunk;
            if (t > 0xffffffffull - kChunk) return "too many steps for one work item";
            C.it_T[it] = (uint32_t)t;
            out.max_T = std::max<uint64_t>(out.max_T, t);
            C.max_T = std::max<uint64_t>(C.max_T, t);
            C.lane_steps += t * kLanes;
        }
        // traceback and hand-over storage
        for (size_t it = 0; it < nit; ++it) {
            uint64_t t = C.it_T[it];
            C.it_ck.push_back(C.ck_words);
            C.it_cb.push_back(C.cb_words);
            C.it_xf.push_back(C.xf_words);
            if (cfg.traceback) {
                C.ck_words += ceil_div(t, (uint64_t)cfg.ckpt) * (uint64_t)wpl * kLanes;
                C.cb_words += (t / kCbitsPer) * kLanes;
            }
            if (C.it_feeds[it]) C.xf_words += 2 * (t / kChunk);
        }
        // traceback order: largest m*n first
        std::vector<size_t> ord(C.tb_pair.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            return pairs[C.tb_pair[a]].m * pairs[C.tb_pair[a]].n >
                   pairs[C.tb_pair[b]].m * pairs[C.tb_pair[b]].n;
        });
        std::vector<uint32_t> tp, ti, tl;
        for (size_t o : ord) {
            tp.push_back(C.tb_pair[o]); ti.push_back(C.tb_item[o]); tl.push_back(C.tb_lane0[o]);
        }
        C.tb_pair.swap(tp); C.tb_item.swap(ti); C.tb_lane0.swap(tl);
        if (cfg.traceback) {
            const uint64_t band = (uint64_t)kLanes * wpl;
            const uint64_t rows = std::max<uint64_t>((uint64_t)std::max(cfg.strip_rows, 1), band);
            C.strip_bands = (uint32_t)ceil_div(rows, band);
            if (cfg.round_bytes) {
                // rounds refill whole items: a strip must not straddle an
                // item boundary, so its band count divides the 64 of an item
                uint32_t sb = 1;
                while (sb < C.strip_bands && sb < (uint32_t)kLanes) sb *= 2;
                C.strip_bands = sb;
            }
            for (size_t t = 0; t < C.tb_pair.size(); ++t) {
                const uint64_t nb = ceil_div(pairs[C.tb_pair[t]].m, band);
                const uint64_t S = ceil_div(nb, (uint64_t)C.strip_bands);
                if (C.n_bands + nb > 0xffffffffull || C.n_strips + S > 0xffffffffull)
                    return "too many traceback bands";
                C.tb_band0.push_back((uint32_t)C.n_bands);
                C.tb_strip0.push_back((uint32_t)C.n_strips);
                C.n_bands += nb;
                C.n_strips += S;
                for (uint64_t s = S; s-- > 0;) {
                    C.sp_t.push_back((uint32_t)t);
                    C.sp_s.push_back((uint32_t)s);
                    if (s + 1 < S) {
                        C.fx_t.push_back((uint32_t)t);
                        C.fx_s.push_back((uint32_t)s);
                    }
                }
                if (S >= 2) C.sl_t.push_back((uint32_t)t);
            }
            // The speculative pass takes its strips longest walk first (rows
            // plus the columns the straight line from (0, 0) to (m, n) crosses
            // in the strip), so that no full strip is left to start late.
            // The strips are independent in this pass.  (Plain mode launches
            // each pair's strips as one range of tickets: pair order kept.)
            if (!cfg.plain) {
                const uint64_t R = (uint64_t)C.strip_bands * band;
                std::vector<uint64_t> est(C.sp_t.size());
                for (size_t k = 0; k < est.size(); ++k) {
                    const PairShape &ps = pairs[C.tb_pair[C.sp_t[k]]];
                    const uint64_t lo = (uint64_t)C.sp_s[k] * R;
                    const uint64_t rows = std::min<uint64_t>(R, ps.m - lo);
                    est[k] = rows + (ps.m ? (uint64_t)((double)ps.n * (double)rows / (double)ps.m) : 0);
                }
                std::vector<size_t> o(est.size());
                std::iota(o.begin(), o.end(), 0);
                std::stable_sort(o.begin(), o.end(), [&](size_t x, size_t y) { return est[x] > est[y]; });
                std::vector<uint32_t> st(o.size()), ss(o.size());
                for (size_t k = 0; k < o.size(); ++k) {
                    st[k] = C.sp_t[o[k]];
                    ss[k] = C.sp_s[o[k]];
                }
                C.sp_t.swap(st);
                C.sp_s.swap(ss);
            }
            if (cfg.round_bytes) {
                std::string why = plan_rounds(pairs, cfg, C);
                if (!why.empty()) return why;
            }
        }
        out.items += nit;
        out.lanes += nit * kLanes;
        out.lane_steps += C.lane_steps;
    }

    // lay out the Y stream: one all-sentinel region per class, then one
    // region per segment
    auto shift_of = [&](int wpl) {
        return raw_stream(cfg.sigma, wpl) ? (uint8_t)0
                                          : (uint8_t)(9 + (wpl == 1 ? 0 : wpl == 2 ? 1 : wpl == 4 ? 2 : 3));
    };
    uint64_t cursor = 0;
    std::vector<uint64_t> class_sent(out.classes.size(), 0);
    for (size_t ci = 0; ci < out.classes.size(); ++ci) {
        const ClassPlan &C = out.classes[ci];
        Segment sg;
        sg.pair = kNoPair;
        sg.pre = 0;
        sg.begin = cursor;
        sg.len = C.max_T + kChunk;
        sg.shift = shift_of(C.wpl);
        class_sent[ci] = cursor;
        cursor += (sg.len + 63) / 64 * 64;
        out.segs.push_back(sg);
    }
    std::vector<uint64_t> seg_col0(np, 0);
    for (const PendingSeg &ps : pend) {
        const ClassPlan &C = out.classes[ps.cls];
        Segment sg;
        sg.pair = ps.pair;
        sg.pre = ps.pre;
        sg.begin = cursor;
        // + one chunk: the fill reads the stream a few steps ahead; with a
        // traceback, whole checkpoint intervals are re-read
        uint64_t Tr = C.it_T[ps.last_item];
        if (cfg.traceback) Tr = ceil_div(Tr, (uint64_t)cfg.ckpt) * cfg.ckpt;
        sg.len = (uint64_t)ps.pre + Tr + kChunk;
        sg.shift = shift_of(C.wpl);
        cursor += (sg.len + 63) / 64 * 64;
        seg_col0[ps.pair] = sg.begin + sg.pre;
        out.segs.push_back(sg);
    }
    out.ys_elems = cursor;
    // lane offsets into the stream
    for (size_t ci = 0; ci < out.classes.size(); ++ci) {
        ClassPlan &C = out.classes[ci];
        for (size_t li = 0; li < C.ln_pair.size(); ++li)
            C.ln_ys[li] = C.ln_pair[li] >= 0 ? seg_col0[C.ln_pair[li]] : class_sent[ci];
    }
    return std::string();
}

std::string check_plan(const std::vector<PairShape> &pairs, const Plan &p) {
    char buf[256];
    const size_t np = pairs.size();
    std::vector<int> seen(np, 0);
    std::vector<int64_t> seg_of(np, -1);
    for (size_t si = 0; si < p.segs.size(); ++si) {
        if (p.segs[si].pair == kNoPair) continue;
        if (p.segs[si].pair >= np) return "segment pair out of range";
        if (seg_of[p.segs[si].pair] >= 0) return "two stream regions for one pair";
        seg_of[p.segs[si].pair] = (int64_t)si;
    }
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        const size_t nit = C.it_T.size();
        if (C.ln_pair.size() != nit * kLanes) return "lane table size";
        for (size_t it = 0; it < nit; ++it) {
            if (C.it_T[it] % kChunk) return "T not a multiple of the chunk";
            if (C.it_prev[it] >= 0 && C.it_prev[it] != (int32_t)it - 1) return "chain not consecutive";
            if (C.it_prev[it] >= 0 && !C.it_feeds[it - 1]) return "chain feed flag";
            if (C.it_prev[it] >= 0 && C.it_T[it] != C.it_T[it - 1]) return "chain step counts differ";
            if (C.it_depth[it] != (C.it_prev[it] >= 0 ? C.it_depth[it - 1] + 1 : 0u))
                return "chain depth";
            for (int l = 0; l < kLanes; ++l) {
                size_t li = it * kLanes + l;
                int32_t pr = C.ln_pair[li];
                if (pr < 0) continue;
                if ((size_t)pr >= np) return "pair index out of range";
                const PairShape &ps = pairs[pr];
                uint64_t W = (ps.m + 63) / 64;
                uint64_t word0 = C.ln_word0[li];
                if (word0 >= W) return "lane holds no word of its pair";
                if (word0 % C.wpl) return "word offset not aligned";
                // the lane below holds the previous words of the same pair,
                // either in this item or in lane 63 of the previous item
                if (word0 > 0) {
                    int32_t below_pair;
                    uint32_t below_word0, below_skew;
                    if (l > 0) {
                        below_pair = C.ln_pair[li - 1];
                        below_word0 = C.ln_word0[li - 1];
                        below_skew = C.ln_skew[li - 1];
                        if (C.ln_skew[li] != below_skew + 1) return "skew step inside an item";
                    } else {
                        if (C.it_prev[it] < 0) return "continuation without a feeding item";
                        size_t lb = (it - 1) * kLanes + kLanes - 1;
                        below_pair = C.ln_pair[lb];
                        below_word0 = C.ln_word0[lb];
                        below_skew = C.ln_skew[lb];
                        if (C.ln_skew[li] != below_skew + kChunk) return "skew step across items";
                    }
                    if (below_pair != pr || below_word0 + C.wpl != word0) return "segment not contiguous";
                } else {
                    if (C.ln_skew[li] != 0) return "segment start with non-zero skew";
                    seen[pr] += 1;
                }
                // every column reached before the item ends
                if ((uint64_t)C.ln_skew[li] + ps.n > C.it_T[it]) {
                    snprintf(buf, sizeof buf, "item %zu lane %d too few steps", it, l);
                    return buf;
                }
                // stream reads stay inside the segment's region
                if (seg_of[pr] < 0) return "segment without a stream region";
                const Segment &sg = p.segs[seg_of[pr]];
                if (C.ln_ys[li] != sg.begin + sg.pre) return "stream offset";
                if (C.ln_skew[li] > sg.pre) return "skew beyond the pre-pad";
                if ((uint64_t)sg.pre + C.it_T[it] + kChunk > sg.len) return "stream region too short";
            }
            // the lane of the pair with the highest word must be the last of
            // its segment: a lane above it holding the same pair is an error
        }
    }
    for (size_t k = 0; k < np; ++k) {
        bool empty = pairs[k].m == 0 || pairs[k].n == 0;
        if (empty && seen[k] != 0) return "empty pair scheduled";
        if (!empty && seen[k] != 1) {
            snprintf(buf, sizeof buf, "pair %zu scheduled %d times", k, seen[k]);
            return buf;
        }
    }
    // every word of every pair is held by exactly one lane
    std::vector<uint64_t> words(np, 0);
    for (const ClassPlan &C : p.classes)
        for (size_t li = 0; li < C.ln_pair.size(); ++li)
            if (C.ln_pair[li] >= 0) {
                const PairShape &ps = pairs[C.ln_pair[li]];
                uint64_t W = (ps.m + 63) / 64;
                words[C.ln_pair[li]] += std::min<uint64_t>(C.wpl, W - C.ln_word0[li]);
            }
    for (size_t k = 0; k < np; ++k)
        if (pairs[k].m && pairs[k].n && words[k] != (pairs[k].m + 63) / 64) return "word coverage";
    // idle lanes read their class's all-sentinel region, long enough for
    // every item of the class
    std::vector<const Segment *> sent;
    for (const Segment &sg : p.segs)
        if (sg.pair == kNoPair) sent.push_back(&sg);
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        for (size_t li = 0; li < C.ln_pair.size(); ++li) {
            if (C.ln_pair[li] >= 0) continue;
            bool ok = false;
            for (const Segment *sg : sent)
                if (sg->begin == C.ln_ys[li] && sg->len >= C.it_T[li / kLanes] + kChunk &&
                    C.ln_skew[li] == 0 &&
                    sg->shift == (raw_stream(p.cfg.sigma, C.wpl) ? 0 : 9 + __builtin_ctz((unsigned)C.wpl)))
                    ok = true;
            if (!ok) return "idle lane without a sentinel region";
        }
    }
    // traceback strips: every strip of every traceback pair has exactly one
    // speculative ticket, every strip below the top one one fix-up ticket,
    // and the band and strip tables tile their arrays in entry order
    for (const ClassPlan &C : p.classes) {
        if (!p.cfg.traceback) break;
        const size_t nt = C.tb_pair.size();
        if (C.tb_band0.size() != nt || C.tb_strip0.size() != nt) return "strip table size";
        const uint64_t band = (uint64_t)kLanes * C.wpl;
        uint64_t b0 = 0, s0 = 0, nseal = 0;
        for (size_t t = 0; t < nt; ++t) {
            const uint64_t nb = (pairs[C.tb_pair[t]].m + band - 1) / band;
            const uint64_t S = (nb + C.strip_bands - 1) / C.strip_bands;
            if (C.tb_band0[t] != b0 || C.tb_strip0[t] != s0) return "strip tables not contiguous";
            b0 += nb;
            s0 += S;
            nseal += S >= 2;
        }
        if (b0 != C.n_bands || s0 != C.n_strips) return "strip totals";
        std::vector<std::vector<uint8_t>> seen_sp(nt), seen_fx(nt);
        for (size_t t = 0; t < nt; ++t) {
            const uint64_t nb = (pairs[C.tb_pair[t]].m + band - 1) / band;
            const uint64_t S = (nb + C.strip_bands - 1) / C.strip_bands;
            seen_sp[t].assign(S, 0);
            seen_fx[t].assign(S, 0);
        }
        if (C.sp_t.size() != C.sp_s.size() || C.fx_t.size() != C.fx_s.size()) return "ticket arrays";
        for (size_t k = 0; k < C.sp_t.size(); ++k) {
            if (C.sp_t[k] >= nt || C.sp_s[k] >= seen_sp[C.sp_t[k]].size()) return "speculative ticket range";
            if (seen_sp[C.sp_t[k]][C.sp_s[k]]++) return "strip walked twice";
        }
        for (size_t k = 0; k < C.fx_t.size(); ++k) {
            if (C.fx_t[k] >= nt || C.fx_s[k] + 1 >= seen_fx[C.fx_t[k]].size()) return "fix-up ticket range";
            if (seen_fx[C.fx_t[k]][C.fx_s[k]]++) return "strip fixed twice";
        }
        if (p.cfg.plain) {
            // plain mode launches the tickets of one entry in a pass as one range
            const auto contiguous = [&](const std::vector<uint32_t> &tk) {
                std::vector<uint8_t> done(nt, 0);
                for (size_t k = 0; k < tk.size(); ++k) {
                    if (k > 0 && tk[k] == tk[k - 1]) continue;
                    if (done[tk[k]]++) return false;
                }
                return true;
            };
            if (!contiguous(C.sp_t) || !contiguous(C.fx_t)) return "plain tickets not contiguous";
        }
        for (size_t t = 0; t < nt; ++t) {
            for (size_t s = 0; s < seen_sp[t].size(); ++s) {
                if (!seen_sp[t][s]) return "strip without a speculative walk";
                if (s + 1 < seen_sp[t].size() && !seen_fx[t][s]) return "strip without a fix-up";
            }
        }
        if (C.sl_t.size() != nseal) return "seal tickets";
        for (size_t k = 0; k < C.sl_t.size(); ++k)
            if (C.sl_t[k] >= nt || seen_sp[C.sl_t[k]].size() < 2) return "seal ticket";
        if (!p.cfg.round_bytes) continue;
        // rounds: every item refilled in exactly one round, within the round
        // capacity, its history inside the round buffer and apart from the
        // other items of its round; chains top-down
        const size_t nit = C.it_T.size();
        const uint32_t R = C.n_rounds;
        if (C.it_round.size() != nit || C.it_rb.size() != nit || C.rd_item_off.size() != R + 1 ||
            C.rd_sp_off.size() != R + 1 || C.rd_fx_off.size() != R + 1 || C.rd_sl_off.size() != R + 1)
            return "round table sizes";
        std::vector<int> refills(nit, 0);
        for (uint32_t r = 0; r < R; ++r) {
            std::vector<std::pair<uint64_t, uint64_t>> iv;
            uint64_t used = 0;
            for (uint32_t k = C.rd_item_off[r]; k < C.rd_item_off[r + 1]; ++k) {
                const uint32_t it = C.rd_items[k];
                if (it >= nit || C.it_round[it] != r) return "round item";
                if (C.it_rcb[it] != 2 * (C.it_rb[it] + item_ck_words(C, it, p.cfg.ckpt)))
                    return "round carry-word offset";
                ++refills[it];
                const uint64_t w = item_round_words(C, it, p.cfg.ckpt);
                iv.push_back({C.it_rb[it], C.it_rb[it] + w});
                used += w;
            }
            if (used * 8 > p.cfg.round_bytes || used > C.round_words) return "round over capacity";
            std::sort(iv.begin(), iv.end());
            for (size_t k = 0; k < iv.size(); ++k) {
                if (iv[k].second > C.round_words) return "item history beyond the round buffer";
                if (k && iv[k].first < iv[k - 1].second) return "item histories overlap";
            }
        }
        for (size_t it = 0; it < nit; ++it) {
            if (refills[it] != 1) return "item not refilled exactly once";
            if (C.it_prev[it] >= 0 && C.it_round[it - 1] < C.it_round[it])
                return "chain item refilled before the item above it";
        }
        // every strip walked speculatively once, in the round of its items;
        // group tops below a pair's top strip start from the strip above;
        // fix-ups for every other strip of a group; one seal per group of
        // two or more strips
        std::vector<std::vector<int>> sp2(nt), fx2(nt), top_of(nt);
        for (size_t t = 0; t < nt; ++t) {
            sp2[t].assign(seen_sp[t].size(), 0);
            fx2[t].assign(seen_sp[t].size(), 0);
            top_of[t].assign(seen_sp[t].size(), -1);
        }
        auto strip_round = [&](size_t t, uint64_t s) {
            return C.it_round[C.tb_item[t] + (C.tb_lane0[t] + s * C.strip_bands) / kLanes];
        };
        for (uint32_t r = 0; r < R; ++r) {
            for (uint32_t k = C.rd_sp_off[r]; k < C.rd_sp_off[r + 1]; ++k) {
                const uint32_t t = C.rd_sp_t[k], sv = C.rd_sp_s[k] & ~kFromAbove;
                if (t >= nt || sv >= sp2[t].size()) return "round speculative ticket range";
                if (strip_round(t, sv) != r) return "strip walked in another round";
                ++sp2[t][sv];
                const bool above = (C.rd_sp_s[k] & kFromAbove) != 0;
                const bool group_top = sv + 1 == sp2[t].size() || strip_round(t, sv + 1) != r;
                if (above != (group_top && sv + 1 < sp2[t].size())) return "round start flag";
            }
            for (uint32_t k = C.rd_fx_off[r]; k < C.rd_fx_off[r + 1]; ++k) {
                const uint32_t t = C.rd_fx_t[k], sv = C.rd_fx_s[k];
                if (t >= nt || sv + 1 >= fx2[t].size()) return "round fix-up ticket range";
                if (strip_round(t, sv) != r || strip_round(t, sv + 1) != r) return "fix-up across rounds";
                ++fx2[t][sv];
            }
            for (uint32_t k = C.rd_sl_off[r]; k < C.rd_sl_off[r + 1]; ++k) {
                const uint32_t t = C.rd_sl_t[k], top = C.rd_sl_top[k], lo = C.rd_sl_lo[k];
                if (t >= nt || top >= sp2[t].size() || lo >= top) return "round seal ticket range";
                if (strip_round(t, top) != r || strip_round(t, lo) != r) return "seal across rounds";
                if (top + 1 < sp2[t].size() && strip_round(t, top + 1) == r) return "seal below a group top";
                if (lo > 0 && strip_round(t, lo - 1) == r) return "seal above a group bottom";
                for (uint32_t q = lo; q <= top; ++q)
                    if (top_of[t][q]++ != -1) return "strip sealed twice";
            }
        }
        for (size_t t = 0; t < nt; ++t)
            for (size_t q = 0; q < sp2[t].size(); ++q) {
                if (sp2[t][q] != 1) return "strip not walked once in the rounds";
                const bool group_top = q + 1 == sp2[t].size() || strip_round(t, q + 1) != strip_round(t, q);
                if (fx2[t][q] != (group_top ? 0 : 1)) return "round fix-ups";
                const bool single = group_top && (q == 0 || strip_round(t, q - 1) != strip_round(t, q));
                if ((top_of[t][q] == -1) != single) return "round seals";
            }
    }
    // regions do not overlap
    std::vector<std::pair<uint64_t, uint64_t>> iv;
    for (const Segment &sg : p.segs) iv.push_back({sg.begin, sg.begin + sg.len});
    std::sort(iv.begin(), iv.end());
    for (size_t k = 1; k < iv.size(); ++k)
        if (iv[k].first < iv[k - 1].second) return "stream regions overlap";
    if (!iv.empty() && iv.back().second > p.ys_elems) return "stream region beyond the stream";
    // ... and tile the stream in whole 64-element blocks, back to back (the
    // stream kernel finds a block's region from a per-block table)
    uint64_t at = 0;
    for (const Segment &sg : p.segs) {
        if (sg.begin != at) return "stream regions not back to back";
        at += (sg.len + 63) / 64 * 64;
    }
    if (at != p.ys_elems) return "stream length";
    return std::string();
}

}  // namespace lcs
