// Admission and continuous-batching policy of the request loop (plain C++,
// no HIP: the device side is an executor passed in, so the policy runs on
// the host with a fake clock in the tests).
//
// Each step at time `now`:
//   1. retire the launch units whose completion the executor reports, giving
//      their bytes back to the HBM budget;
//   2. admit pending jobs in arrival (FIFO) order while the in-flight bytes
//      (input + output of every admitted, unfinished job) stay within the
//      budget -- the head of the queue blocks the rest until it fits;
//   3. split the jobs admitted in this step into launch units: with batching,
//      the small jobs of each kind share one unit (one launch per element size
//      or dtype) and every large job is a unit of its own (it is
//      bandwidth-bound and gains nothing from sharing a launch) -- unless jobs
//      are left waiting, when the large jobs of a kind share a unit too (then
//      launches are the scarce resource); a shared unit holds at most
//      `max_per_kind` jobs of a kind (0: no limit); without batching, one unit
//      per job;
//   4. launch every unit at once, each with its own completion event: on the
//      next of K streams, or -- with the large-job lane -- every unit that
//      holds a large job on stream 0, in admission order, and the others on
//      streams 1..K-1 in turn.  Large jobs then run one after another at the
//      full bandwidth instead of sharing it, which shortens the tail of the
//      latency distribution (its top percent is made of the largest jobs),
//      while small jobs never queue behind them.
// Jobs that arrive while others run join the next unit as soon as budget
// frees up, and units on different streams overlap on the device.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace xtr {
namespace srv {

struct Pending {
    int64_t id;        // job index in submission order
    int64_t bytes;     // input + output bytes
    int32_t kind;      // 0 transpose, 1 sum
    int32_t _pad;
};

// Launch units of the jobs admitted in one step (order of admission kept).
inline void make_units(const std::vector<Pending> &group, bool batching, bool backlog,
                       int64_t small_bytes, int max_per_kind,
                       std::vector<std::vector<Pending>> &units) {
    units.clear();
    if (!batching) {
        for (const Pending &p : group) units.push_back({p});
        return;
    }
    int shared[2][2] = {{-1, -1}, {-1, -1}};   // [kind][small] -> open unit index
    int count[2][2] = {{0, 0}, {0, 0}};        // jobs of that kind in the open unit
    for (const Pending &p : group) {
        const bool small = p.bytes < small_bytes;
        if (small || backlog) {
            const int k = p.kind & 1, c = small ? 1 : 0;
            int &u = shared[k][c];
            if (u < 0 || (max_per_kind > 0 && count[k][c] >= max_per_kind)) {
                u = (int)units.size();
                count[k][c] = 0;
                units.emplace_back();
            }
            units[u].push_back(p);
            count[k][c]++;
        } else {
            units.push_back({p});
        }
    }
}

// Stream of a unit: with the large-job lane (and at least two streams), a
// unit that holds a job of at least small_bytes goes to stream 0 and the
// others take streams 1..K-1 in turn; else every unit takes the next stream.
inline int pick_stream(const std::vector<Pending> &unit, bool big_lane, int nstreams,
                       int64_t small_bytes, int &next_small, int &next_any) {
    if (big_lane && nstreams >= 2) {
        for (const Pending &p : unit)
            if (p.bytes >= small_bytes) return 0;
        const int s = 1 + next_small;
        next_small = (next_small + 1) % (nstreams - 1);
        return s;
    }
    const int s = next_any;
    next_any = (next_any + 1) % nstreams;
    return s;
}

// Exec: int64_t launch(const std::vector<Pending> &unit, int stream) returns a
// handle (>= 0) or -1 on failure; int64_t done(int64_t handle) returns the
// completion time (ns) or -1 while running.
template <class Exec> class Scheduler {
  public:
    Scheduler(Exec &ex, int64_t budget, bool batching, int nstreams, int64_t small_bytes,
              bool big_lane = false, int max_per_kind = 0)
        : ex_(ex), budget_(budget), batching_(batching), nstreams_(nstreams),
          small_(small_bytes), big_lane_(big_lane), max_per_kind_(max_per_kind) {}

    void arrive(const Pending &p) { pending_.push_back(p); }

    // One pass at time `now`; completion times go to done[id] (failed
    // launches: -2) and the ids of the jobs that finished to `finished`.
    // Returns true if it launched anything.
    bool step(int64_t now, std::vector<int64_t> &done, std::vector<int64_t> &finished) {
        (void)now;
        for (size_t i = 0; i < inflight_.size();) {
            const int64_t t = ex_.done(inflight_[i].handle);
            if (t < 0) {
                i++;
                continue;
            }
            for (const Pending &p : inflight_[i].jobs) {
                done[p.id] = t;
                finished.push_back(p.id);
                used_ -= p.bytes;
            }
            inflight_[i] = std::move(inflight_.back());
            inflight_.pop_back();
        }
        group_.clear();
        while (!pending_.empty() && used_ + pending_.front().bytes <= budget_) {
            used_ += pending_.front().bytes;
            group_.push_back(pending_.front());
            admit_order.push_back(pending_.front().id);
            pending_.pop_front();
        }
        if (used_ > max_used) max_used = used_;
        if (group_.empty()) return false;
        make_units(group_, batching_, !pending_.empty(), small_, max_per_kind_, units_);
        for (auto &u : units_) {
            const int si = pick_stream(u, big_lane_, nstreams_, small_, next_small_, si_);
            const int64_t h = ex_.launch(u, si);
            units++;
            if (h < 0) {   // nothing of the unit runs: its jobs fail now
                for (const Pending &p : u) {
                    done[p.id] = -2;
                    finished.push_back(p.id);
                    used_ -= p.bytes;
                }
                failed += (int64_t)u.size();
                continue;
            }
            inflight_.push_back(Unit{std::move(u), h});
        }
        return true;
    }

    bool idle() const { return pending_.empty() && inflight_.empty(); }
    bool has_pending() const { return !pending_.empty(); }
    int64_t used() const { return used_; }

    int64_t max_used = 0, units = 0, failed = 0;
    std::vector<int64_t> admit_order;

  private:
    struct Unit {
        std::vector<Pending> jobs;
        int64_t handle;
    };
    Exec &ex_;
    int64_t budget_, used_ = 0;
    bool batching_;
    int nstreams_, si_ = 0, next_small_ = 0;
    int64_t small_;
    bool big_lane_;
    int max_per_kind_;
    std::deque<Pending> pending_;
    std::vector<Unit> inflight_;
    std::vector<Pending> group_;
    std::vector<std::vector<Pending>> units_;
};

}  // namespace srv
}  // namespace xtr
