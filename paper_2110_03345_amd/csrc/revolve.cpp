// Binomial checkpointing schedules; see revolve.h for the recurrences.
#include "revolve.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

namespace stride {

namespace {

constexpr long long kSat = (long long)4e18;

// beta(c, t) = (c + t)! / (c! t!), saturating at kSat.
long long beta(long long c, long long t)
{
    long long r = 1;
    for (long long i = 1; i <= t; ++i) {
        // r * (c + i) / i is the exact binomial C(c + i, i)
        if (r > kSat / (c + i))
            return kSat;
        r = r * (c + i) / i;
    }
    return r;
}

struct Generator {
    std::vector<Action>& out;
    std::unordered_map<long long, int> memo;
    int cur = 0;

    explicit Generator(std::vector<Action>& o) : out(o) {}

    // An optimal first checkpoint: the target cost C(l, s) is known in closed
    // form, so search outward from the repetition-count estimate and stop at
    // the first m that attains it.
    int split(int l, int s)
    {
        if (s >= l - 1)
            return 1;   // every state can be kept: store each one in turn
        long long key = (long long)l * 1000003LL + s;
        auto it = memo.find(key);
        if (it != memo.end())
            return it->second;
        const long long target = revolve_cost(l, s);
        long long t = 1;
        while (beta(s + 1, t) < l)
            ++t;
        long long guess = std::max<long long>(t >= 2 ? beta(s + 1, t - 2) : 1, l - beta(s, t - 1));
        guess = std::min<long long>(std::max<long long>(guess, 1), l - 1);
        auto cost = [&](long long m) { return m + revolve_cost(l - m, s - 1) + revolve_cost(m, s); };
        int bm = -1;
        for (long long d = 0; bm < 0 && d < l; ++d) {
            if (guess - d >= 1 && cost(guess - d) == target)
                bm = (int)(guess - d);
            else if (guess + d <= l - 1 && cost(guess + d) == target)
                bm = (int)(guess + d);
        }
        if (bm < 0)
            bm = (int)guess;   // unreachable: the closed form is attained by some m
        memo.emplace(key, bm);
        return bm;
    }

    void go(int a, int i)
    {
        if (cur == i)
            return;
        if (cur > i || cur < a) {
            out.push_back({Act::Restore, a});
            cur = a;
        }
        if (cur < i) {
            out.push_back({Act::Advance, i});
            cur = i;
        }
    }

    // Precondition: x_a is stored.  Emits Reverse(b-1), ..., Reverse(a).
    void rev(int a, int b, int s)
    {
        int l = b - a;
        if (l == 1) {
            go(a, a);
            out.push_back({Act::Reverse, a});
            return;
        }
        if (s == 0) {
            for (int i = b - 1; i >= a; --i) {
                go(a, i);
                out.push_back({Act::Reverse, i});
            }
            return;
        }
        int m = a + split(l, s);
        go(a, m);
        out.push_back({Act::Store, m});
        rev(m, b, s - 1);
        out.push_back({Act::Free, m});
        rev(a, m, s);
    }
};

}  // namespace

int snaps_search(int nt, long long fields);

long long revolve_cost(long long l, long long s)
{
    if (l <= 1)
        return 0;
    if (s <= 0)
        return l * (l - 1) / 2;
    long long t = 1;
    while (beta(s + 1, t) < l)
        ++t;
    return t * l - beta(s + 2, t - 1);
}

std::vector<Action> revolve_schedule(int nt, int snaps)
{
    std::vector<Action> out;
    if (nt < 1)
        return out;
    if (snaps < 0)
        snaps = 0;
    if (snaps > nt)
        snaps = nt;
    Generator g(out);
    out.push_back({Act::Store, 0});
    g.cur = 0;
    g.rev(0, nt, snaps);
    out.push_back({Act::Free, 0});
    return out;
}

ScheduleStats schedule_stats(const std::vector<Action>& sched)
{
    ScheduleStats st{0, 0, 0};
    std::vector<int> ref;
    std::vector<int> freelist;
    int alive = 0;
    auto alloc = [&]() {
        int f;
        if (!freelist.empty()) {
            f = freelist.back();
            freelist.pop_back();
        } else {
            f = (int)ref.size();
            ref.push_back(0);
        }
        ref[f] = 1;
        ++alive;
        st.peak_fields = std::max(st.peak_fields, alive);
        return f;
    };
    auto release = [&](int f) {
        if (--ref[f] == 0) {
            --alive;
            freelist.push_back(f);
        }
    };
    std::unordered_map<int, std::pair<int, int>> snaps;
    int cur = alloc(), prev = alloc(), idx = 0;
    for (const Action& a : sched) {
        switch (a.type) {
        case Act::Advance:
            while (idx < a.step) {
                int out;
                if (ref[prev] == 1) {
                    out = prev;
                } else {
                    out = alloc();
                    release(prev);
                }
                prev = cur;
                cur = out;
                ++idx;
                ++st.forward_steps;
            }
            break;
        case Act::Store:
            snaps[a.step] = {cur, prev};
            ++ref[cur];
            ++ref[prev];
            st.max_snaps = std::max(st.max_snaps, (int)snaps.size());
            break;
        case Act::Free: {
            auto it = snaps.find(a.step);
            if (it != snaps.end()) {
                release(it->second.first);
                release(it->second.second);
                snaps.erase(it);
            }
            break;
        }
        case Act::Restore: {
            auto it = snaps.find(a.step);
            release(cur);
            release(prev);
            cur = it->second.first;
            prev = it->second.second;
            ++ref[cur];
            ++ref[prev];
            idx = a.step;
            break;
        }
        case Act::Reverse:
            break;
        }
    }
    return st;
}

int snaps_for_fields(int nt, long long fields)
{
    if (nt < 1 || fields < 3)
        return -1;
    // the answer depends on (nt, fields) only: cache it for repeated solves
    static std::mutex mu;
    static std::map<std::pair<int, long long>, int> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({nt, fields});
        if (it != cache.end())
            return it->second;
    }
    int s = snaps_search(nt, fields);
    std::lock_guard<std::mutex> lk(mu);
    cache[{nt, fields}] = s;
    return s;
}

std::shared_ptr<const CachedSchedule> cached_schedule(int nt, int snaps)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::shared_ptr<const CachedSchedule>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({nt, snaps});
        if (it != cache.end())
            return it->second;
    }
    auto cs = std::make_shared<CachedSchedule>();
    cs->actions = revolve_schedule(nt, snaps);
    cs->stats = schedule_stats(cs->actions);
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() > 64)
        cache.clear();
    cache[{nt, snaps}] = cs;
    return cs;
}

int snaps_search(int nt, long long fields)
{
    auto fits = [&](int s) { return schedule_stats(revolve_schedule(nt, s)).peak_fields <= fields; };
    if (!fits(0))
        return -1;
    if (fits(nt))
        return nt;
    int lo = 0, hi = nt;   // fits(lo), !fits(hi)
    while (hi - lo > 1) {
        int mid = lo + (hi - lo) / 2;
        if (fits(mid))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace stride
