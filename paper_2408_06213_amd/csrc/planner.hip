// Host-side planning: the per-die cost model of Sec. 6.1, the batch-size
// thresholds n_k it implies (Table 2), and schedules derived from them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "brr.h"
#include "internal.hpp"

namespace {

typedef unsigned __int128 u128;

// n^(falling k) as an exact integer, or 0 when it exceeds 2^L.
u128 falling_le(uint64_t n, uint32_t k, uint32_t L)
{
    const u128 lim = (u128)1 << L;
    u128 p = 1;
    for (uint32_t l = 0; l < k; ++l) {
        if (n < l + 1) return 0;
        p *= (u128)(n - l);
        if (p > lim) return 0;
    }
    return p;
}

double two_pow(uint32_t L) { return std::ldexp(1.0, (int)L); }

// Expected cost per die of batches of k at size n (Sec. 6.1): every roll
// costs one word and k multiplies, 1/(1 - p2) rolls on average, and with
// probability p1 the product and the threshold cost k - 1 multiplies and one
// division, where p1 = n^(falling k) / 2^L and p2 = (2^L mod n^(falling k)) / 2^L.
double cost_per_die(uint64_t n, uint32_t k, uint32_t L, double c_rng, double c_div)
{
    const u128 b = falling_le(n, k, L);
    if (b == 0) return INFINITY;
    const double scale = two_pow(L);
    const double p1 = (double)b / scale;
    const double p2 = (double)((((u128)1) << L) % b) / scale;
    return ((c_rng + k) / (1.0 - p2) + (c_div + k - 1) * p1) / k;
}

// Upper bound of cost(k, n) (p2 < p1) and lower bound of cost(k-1, n)
// (p2 >= 0), both non-decreasing in n.
double cost_upper(uint64_t n, uint32_t k, uint32_t L, double c_rng, double c_div)
{
    const u128 b = falling_le(n, k, L);
    if (b == 0) return INFINITY;
    const double p1 = (double)b / two_pow(L);
    if (p1 >= 1.0) return INFINITY;
    return ((c_rng + k) / (1.0 - p1) + (c_div + k - 1) * p1) / k;
}

// n_k (Table 2): the largest n such that a batch of k costs less per die
// than a batch of k - 1 at every size from k up to n. Sizes where the
// comparison cannot fail (the upper bound of cost(k) below the smallest
// cost(k-1)) are skipped; the rest are scanned one by one with the exact
// costs.
uint64_t threshold_nk(uint32_t k, uint32_t L, double c_rng, double c_div)
{
    const double floor_prev = (c_rng + (k - 1)) / (double)(k - 1);
    uint64_t lo = k, hi = k;
    while (cost_upper(hi, k, L, c_rng, c_div) < floor_prev) {
        lo = hi;
        hi = hi * 2;
        if (hi > (1ull << 62)) break;
    }
    while (hi - lo > 1) { // the largest n with the safe bound holding
        const uint64_t mid = lo + (hi - lo) / 2;
        if (cost_upper(mid, k, L, c_rng, c_div) < floor_prev)
            lo = mid;
        else
            hi = mid;
    }
    for (uint64_t n = lo;; ++n) {
        const double ck = cost_per_die(n, k, L, c_rng, c_div);
        const double cp = cost_per_die(n, k - 1, L, c_rng, c_div);
        if (!(ck < cp)) return n - 1;
        if (n == ~0ull) return n;
    }
}

// The cost model with p2 replaced by its mean p1 / 2 (2^L mod b is spread
// over [0, b)): smooth in n, so the first size where k dice stop paying off
// is found by bisection instead of a scan.
double smooth_cost(uint64_t n, uint32_t k, uint32_t L, double c_rng, double c_div)
{
    const u128 b = falling_le(n, k, L);
    if (b == 0) return INFINITY;
    const double p1 = (double)b / two_pow(L);
    return ((c_rng + k) / (1.0 - p1 / 2) + (c_div + k - 1) * p1) / k;
}

uint64_t threshold_nk_smooth(uint32_t k, uint32_t L, double c_rng, double c_div)
{
    auto ok = [&](uint64_t n) {
        return smooth_cost(n, k, L, c_rng, c_div) < smooth_cost(n, k - 1, L, c_rng, c_div);
    };
    if (!ok(k)) return k - 1;
    uint64_t lo = k, hi = k;
    while (ok(hi)) {
        lo = hi;
        if (hi > (1ull << 62)) return hi;
        hi *= 2;
    }
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        (ok(mid) ? lo : hi) = mid;
    }
    return lo;
}

uint64_t floor_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p <= x / 2) p *= 2;
    return p;
}

} // namespace

extern "C" {

double brr_cost_per_die(uint64_t n, uint32_t k, uint32_t L, double c_rng, double c_div)
{
    if (k == 0 || L == 0 || L > 64) return NAN;
    return cost_per_die(n, k, L, c_rng, c_div);
}

brr_status brr_cost_thresholds(uint32_t L, uint32_t kmax, double c_rng, double c_div,
                               uint64_t *out_nk)
{
    if (!out_nk || L < 8 || L > 64 || kmax < 2 || kmax > BRR_MAX_K) return BRR_EINVAL;
    out_nk[0] = out_nk[1] = 0;
    for (uint32_t k = 2; k <= kmax; ++k) {
        // the exact scan takes seconds for k = 2 at L = 64: remember results
        static std::mutex mu;
        static std::map<std::tuple<uint32_t, uint32_t, double, double>, uint64_t> memo;
        const auto key = std::make_tuple(k, L, c_rng, c_div);
        {
            std::lock_guard<std::mutex> lock(mu);
            auto it = memo.find(key);
            if (it != memo.end()) {
                out_nk[k] = it->second;
                continue;
            }
        }
        const uint64_t v = threshold_nk(k, L, c_rng, c_div);
        std::lock_guard<std::mutex> lock(mu);
        memo[key] = out_nk[k] = v;
    }
    return BRR_OK;
}

brr_status brr_schedule_from_costs(uint32_t kmax, double c_rng, double c_div, int pow2,
                                   brr_schedule *out)
{
    if (!out || kmax < 1 || kmax > BRR_MAX_K) return BRR_EINVAL;
    brr_schedule s;
    std::memset(&s, 0, sizeof s);
    const uint32_t L = (pow2 & BRR_COSTS_L32) ? 32 : 64;
    if (kmax == 1) {
        const brr_status st = brr_schedule_paper(1, out);
        if (L == 32) out->words = BRR_WORDS_PHILOX32;
        return st;
    }
    uint64_t nk[BRR_MAX_K + 1];
    if (pow2 & BRR_COSTS_SMOOTH) {
        for (uint32_t k = 2; k <= kmax; ++k) nk[k] = threshold_nk_smooth(k, L, c_rng, c_div);
    } else {
        const brr_status st = brr_cost_thresholds(L, kmax, c_rng, c_div, nk);
        if (st != BRR_OK) return st;
    }
    // one die while more than n_2 elements remain, then k dice while more than
    // n_{k+1}, the last k down to n_above = k; guards u_k = n_k^k (a power of
    // two when n_k is one, as in the paper's shuffle_6)
    uint64_t above[BRR_MAX_K + 2];
    for (uint32_t k = 2; k <= kmax; ++k)
        above[k] = std::max<uint64_t>(k, (pow2 & BRR_COSTS_POW2) ? floor_pow2(nk[k]) : nk[k]);
    // thresholds must not increase with k
    for (uint32_t k = 3; k <= kmax; ++k)
        if (above[k] > above[k - 1]) above[k] = above[k - 1];
    s.nsteps = 0;
    s.step[s.nsteps++] = brr_step{above[2], 1, 0, 0};
    for (uint32_t k = 2; k <= kmax; ++k) {
        const uint64_t lim = (k < kmax) ? above[k + 1] : k;
        const uint64_t top = above[k];
        u128 u = 1;
        for (uint32_t l = 0; l < k; ++l) u *= top;
        const uint64_t u0 = (u >= ((u128)1 << L)) ? 0 : (uint64_t)u; // 0: exact product
        s.step[s.nsteps++] = brr_step{std::max<uint64_t>(lim, k - 1), k, 0, u0};
    }
    s.tail = 1;
    // the last batch has at most kmax - 1 dice below kmax + 1 elements
    u128 tail = 1;
    for (uint32_t v = 2; v <= kmax; ++v) tail *= v;
    s.u_tail = (uint64_t)tail;
    s.words = (L == 32) ? BRR_WORDS_PHILOX32 : BRR_WORDS_PHILOX64;
    *out = s;
    return BRR_OK;
}

} // extern "C"
