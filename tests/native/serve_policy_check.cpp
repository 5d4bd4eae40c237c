// Host check of the native request loop's policy (serve_policy.h) with a fake
// clock and a fake executor that completes a unit a fixed latency plus its
// bytes at a set bandwidth after launch:
//   * the in-flight bytes never exceed the budget, and reach it under load;
//   * admission is in arrival (FIFO) order, every job completes once, after
//     its arrival;
//   * the batching rule: small jobs of a kind share a unit, a large job is a
//     unit of its own unless jobs are left waiting; without batching every
//     unit holds one job;
//   * a launch that fails marks its jobs failed (-2) and frees their budget;
//   * with a cap of jobs per kind, no unit holds more than the cap;
//   * with the large-job lane, every unit holding a large job goes to stream
//     0 (and only those), in admission order.
#include "../../paper_2605_13864_amd/csrc/serve_policy.h"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

using xtr::srv::Pending;

static int failures = 0;
#define CHECK(c, ...)                                                        \
    do {                                                                     \
        if (!(c)) {                                                          \
            if (++failures < 20) {                                           \
                std::printf("FAIL line %d: ", __LINE__);                     \
                std::printf(__VA_ARGS__);                                    \
                std::printf("\n");                                           \
            }                                                                \
        }                                                                    \
    } while (0)

struct FakeExec {
    int64_t *clock;
    double bytes_per_ns;
    int fail_every = 0;                         // every k-th launch fails (0: never)
    std::vector<int64_t> t_done;
    std::vector<std::vector<Pending>> launched;
    std::vector<int> stream_of;
    int64_t calls = 0;
    int64_t launch(const std::vector<Pending> &u, int si) {
        calls++;
        stream_of.push_back(si);
        if (fail_every && calls % fail_every == 0) return -1;
        int64_t b = 0;
        for (const Pending &p : u) b += p.bytes;
        t_done.push_back(*clock + 5000 + (int64_t)(b / bytes_per_ns));
        launched.push_back(u);
        return (int64_t)t_done.size() - 1;
    }
    int64_t done(int64_t h) { return *clock >= t_done[h] ? t_done[h] : -1; }
};

struct Arrival {
    int64_t t;
    Pending p;
};

// a Poisson-like stream with sizes spread over six orders of magnitude
static std::vector<Arrival> stream(int n, unsigned seed, double mean_gap_ns) {
    std::vector<Arrival> a;
    srand(seed);
    double t = 0;
    for (int i = 0; i < n; i++) {
        t += mean_gap_ns * (0.05 + 1.9 * (rand() / (double)RAND_MAX));
        const int kind = rand() % 2;
        const int64_t bytes = (int64_t)1 << (10 + rand() % 17);   // 1 KiB .. 64 MiB
        a.push_back(Arrival{(int64_t)t, Pending{i, bytes, kind, 0}});
    }
    return a;
}

static void run(const char *name, bool batching, int64_t budget, double gbs, int fail_every,
                bool big_lane = false, int cap = 0, double gap_ns = 50000.0) {
    int64_t clock = 0;
    FakeExec ex{&clock, gbs, fail_every};
    const int64_t small = 4 << 20;
    const int nstreams = 3;
    xtr::srv::Scheduler<FakeExec> sch(ex, budget, batching, nstreams, small, big_lane, cap);
    auto arr = stream(20000, 7, gap_ns);
    std::vector<int64_t> done(arr.size(), -1), fin;
    size_t next = 0;
    int64_t max_used = 0, steps = 0;
    std::map<int64_t, int> finished_count;
    while (next < arr.size() || !sch.idle()) {
        while (next < arr.size() && arr[next].t <= clock) sch.arrive(arr[next++].p);
        const size_t before = ex.launched.size();
        const bool backlog_before = false;
        (void)backlog_before;
        fin.clear();
        sch.step(clock, done, fin);
        for (int64_t id : fin) finished_count[id]++;
        // units launched in this step
        for (size_t u = before; u < ex.launched.size(); u++) {
            const auto &unit = ex.launched[u];
            if (!batching) CHECK(unit.size() == 1, "%s: unit of %zu jobs without batching", name, unit.size());
            if (batching && !sch.has_pending() && unit.size() > 1)
                for (const Pending &p : unit)
                    CHECK(p.bytes < small, "%s: large job shared a unit with no backlog", name);
            for (const Pending &p : unit) CHECK(p.kind == unit[0].kind, "%s: kinds mixed in a unit", name);
            if (cap > 0) CHECK((int)unit.size() <= cap, "%s: unit of %zu jobs > cap %d", name, unit.size(), cap);
            bool large = false;
            for (const Pending &p : unit) large |= p.bytes >= small;
            const int si = ex.stream_of[u];
            CHECK(si >= 0 && si < nstreams, "%s: stream %d", name, si);
            if (big_lane) CHECK((si == 0) == large, "%s: unit (large %d) on stream %d", name, (int)large, si);
        }
        if (sch.used() > max_used) max_used = sch.used();
        CHECK(sch.used() <= budget, "%s: %lld bytes in flight > budget", name, (long long)sch.used());
        clock += 20000;
        CHECK(++steps < 100000000, "%s: no progress", name);
        if (failures > 20) break;
    }
    for (size_t i = 0; i < arr.size(); i++) {
        CHECK(done[i] != -1, "%s: job %zu never finished", name, i);
        CHECK(finished_count[(int64_t)i] == 1, "%s: job %zu finished %d times", name, i,
              finished_count[(int64_t)i]);
        if (done[i] >= 0) CHECK(done[i] >= arr[i].t, "%s: job %zu done before arrival", name, i);
    }
    for (size_t i = 0; i < sch.admit_order.size(); i++)
        CHECK(sch.admit_order[i] == (int64_t)i, "%s: admission out of arrival order", name);
    CHECK(sch.max_used == max_used && max_used <= budget, "%s: max in flight", name);
    int64_t failed = 0;
    for (int64_t d : done) failed += d == -2;
    CHECK(failed == sch.failed, "%s: failed count", name);
    if (fail_every) CHECK(failed > 0, "%s: no failed launch", name);
    else CHECK(failed == 0, "%s: unexpected failures", name);
    int64_t maxu = 0;
    for (const auto &u : ex.launched) maxu = (int64_t)u.size() > maxu ? (int64_t)u.size() : maxu;
    std::printf("%-36s largest unit %3lld  units %7lld  launches %7lld  max in flight %6.1f MiB of %6.1f  failed %lld\n",
                name, (long long)maxu, (long long)sch.units, (long long)ex.calls, max_used / 1048576.0,
                budget / 1048576.0, (long long)failed);
}

int main() {
    run("batching, idle device", true, (int64_t)64 << 30, 5000.0, 0);
    run("batching, tight budget", true, (int64_t)96 << 20, 5000.0, 0);
    run("batching, slow device (backlog)", true, (int64_t)1 << 30, 20.0, 0);
    run("one launch per job", false, (int64_t)1 << 30, 20.0, 0);
    run("batching, failing launches", true, (int64_t)1 << 30, 500.0, 7);
    run("batching, large-job lane", true, (int64_t)1 << 30, 20.0, 0, true);
    run("batching, 24 jobs per kind (graphs)", true, (int64_t)1 << 30, 500.0, 0, false, 24, 200.0);
    run("lane + cap, tight budget", true, (int64_t)96 << 20, 500.0, 0, true, 24, 200.0);
    std::printf("%s\n", failures ? "FAILED" : "serving policy ok");
    return failures ? 1 : 0;
}
