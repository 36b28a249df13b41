// Role lock of a table across host threads and streams (Sec. 3.5, the three operation groups and
// their compatibility table; Sec. 4.4, the host/device two-layer lock).
//
// Every call on a table belongs to a role: reader (find, contains, find_ptr, size, export),
// updater (assign, assign_scores) or inserter (insert_or_assign, insert_and_evict,
// find_or_insert, erase).  Calls are admitted in arrival order into groups.  A group holds calls
// of one role that may run at the same time: readers with readers and updaters with updaters
// under the triple-group rule; readers only under the reader/writer rule that the paper's
// ablation compares against.  An inserter (and, under the reader/writer rule, an updater) is a
// group of its own.
//
// The device-side half of the lock is a stream dependency, not a flag polled by kernels: every
// call records an event on its stream after its kernels, and a call of a new group makes its
// stream wait for the events of the group before it.  A group keeps one event per stream (the
// latest: stream order implies the earlier ones), so a long-lived group holds at most one
// event per stream that used it.  Calls of one group therefore overlap on the GPU, and any two
// calls of different groups run in admission order, whatever streams they use.  The host never
// waits for the GPU: it blocks only while an admitted call of the group that is closing is
// still enqueueing its kernels.  The lock keeps events recorded on the callers' streams until
// later calls no longer need them, and it may query or wait on them then; so before a stream
// that made calls under the lock is destroyed, the caller synchronizes it and resets the lock
// (reset() forgets every event it holds).
//
// The lock is a template over its event backend so that the host logic can be tested without a
// GPU: the backend provides Event, Stream, make(), record(e, s) and wait(s, e) (both returning
// false on failure), done(e) and destroy(e).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

namespace cskv {

enum Role { kReader = 0, kUpdater = 1, kInserter = 2 };
enum LockMode { kLockNone = 0, kLockTripleGroup = 1, kLockReaderWriter = 2 };

// may calls of roles a and b belong to one group?
inline bool roles_compatible(int mode, int a, int b) {
    if (a != b) return false;
    return mode == kLockTripleGroup ? a != kInserter : a == kReader;
}

template <class B>
class RoleLock {
  public:
    using Event = typename B::Event;
    using Stream = typename B::Stream;

    struct Group {
        int role = 0;
        uint64_t seq = 0;      // admission order of groups
        int pending = 0;       // admitted calls that have not recorded their event yet
        bool open = true;      // false once a call of another role waits behind it
        std::vector<std::pair<Stream, Event>> events;  // the latest event of each stream
        Group* prev = nullptr;  // the group before; complete (no pending call) once this exists
    };
    struct Ticket {
        Group* g = nullptr;
        uint64_t seq = 0;
        bool ok = true;  // every wait was enqueued
    };

    explicit RoleLock(B backend = B()) : b_(backend) {}
    RoleLock(const RoleLock&) = delete;
    RoleLock& operator=(const RoleLock&) = delete;
    ~RoleLock() {
        std::lock_guard<std::mutex> lk(m_);
        drain_locked();
    }

    int mode() const { return mode_; }
    // set (and reset) while no call is in flight on the table
    bool set_mode(int m) {
        if (!reset()) return false;
        std::lock_guard<std::mutex> lk(m_);
        mode_ = m;
        return true;
    }

    // forgets every event the lock holds and the groups (the caller has synchronized the streams
    // that recorded them); false (and nothing done) while a call is admitted or queued
    bool reset() {
        std::lock_guard<std::mutex> lk(m_);
        if (!q_.empty() || (cur_ && cur_->pending)) return false;
        drain_locked();
        cur_.reset();
        prev_.reset();
        return true;
    }

    // admits a call of `role` whose kernels go to stream s; s is made to wait for the group before
    Ticket acquire(int role, Stream s) {
        std::unique_lock<std::mutex> lk(m_);
        Waiter w{role, nullptr};
        if (q_.empty() && cur_ && cur_->open && roles_compatible(mode_, cur_->role, role)) {
            join(&w, cur_.get());
        } else {
            q_.push_back(&w);
            pump();
            cv_.wait(lk, [&] { return w.g != nullptr; });
        }
        Group* g = w.g;
        const Group* before = g->prev;  // immutable from here on
        lk.unlock();
        bool ok = true;
        if (before)
            for (const auto& se : before->events) ok = b_.wait(s, se.second) && ok;
        return Ticket{g, g->seq, ok};
    }

    // ends a call: records its event on s (after the kernels it enqueued); false if the record
    // failed (the group then keeps no event for this call)
    bool release(const Ticket& t, Stream s) {
        Event e;
        {
            std::lock_guard<std::mutex> lk(m_);
            e = take_event();
        }
        const bool ok = b_.record(e, s);
        std::lock_guard<std::mutex> lk(m_);
        if (ok) {
            // nobody waits on the running group's events yet: a stream's older event is superseded
            bool replaced = false;
            for (auto& se : t.g->events)
                if (se.first == s) {
                    retired_.push_back(se.second);
                    se.second = e;
                    replaced = true;
                    break;
                }
            if (!replaced) t.g->events.emplace_back(s, e);
        } else {
            free_.push_back(e);
        }
        --t.g->pending;
        pump();
        return ok;
    }

  private:
    struct Waiter {
        int role;
        Group* g;
    };

    void join(Waiter* w, Group* g) {
        ++g->pending;
        w->g = g;
    }

    // admits queued calls in order (lock held)
    void pump() {
        while (!q_.empty()) {
            Waiter* h = q_.front();
            if (cur_ && cur_->open && roles_compatible(mode_, cur_->role, h->role)) {
                join(h, cur_.get());
                q_.pop_front();
                continue;
            }
            if (cur_ && cur_->pending > 0) break;  // its event list is not final yet
            start_group(h->role);
            join(h, cur_.get());
            q_.pop_front();
        }
        if (!q_.empty() && cur_) cur_->open = false;  // later arrivals queue behind the waiting call
        cv_.notify_all();
    }

    void start_group(int role) {
        // the group before the current one was waited for by the current one's calls, all of
        // which have enqueued their waits (the current group has no pending call): retire it
        if (prev_) retire(prev_->events);
        if (cur_) cur_->prev = nullptr;
        prev_ = std::move(cur_);
        cur_.reset(new Group());
        cur_->role = role;
        cur_->seq = ++seq_;
        cur_->prev = prev_.get();
    }

    Event take_event() {
        // retired events complete roughly in the order they retired: recycle from the front
        for (int k = 0; k < 64 && !retired_.empty() && b_.done(retired_.front()); ++k) {
            free_.push_back(retired_.front());
            retired_.pop_front();
        }
        if (free_.empty()) return b_.make();
        Event e = free_.back();
        free_.pop_back();
        return e;
    }

    void retire(std::vector<std::pair<Stream, Event>>& ev) {
        for (const auto& se : ev) retired_.push_back(se.second);
        ev.clear();
    }

    void drain_locked() {
        if (prev_) retire(prev_->events);
        if (cur_) retire(cur_->events);
        for (const Event& e : retired_) b_.destroy(e);  // a pending event may be destroyed
        for (const Event& e : free_) b_.destroy(e);
        retired_.clear();
        free_.clear();
    }

    B b_;
    std::mutex m_;
    std::condition_variable cv_;
    int mode_ = kLockNone;
    uint64_t seq_ = 0;
    std::unique_ptr<Group> cur_, prev_;
    std::deque<Waiter*> q_;
    std::vector<Event> free_;
    std::deque<Event> retired_;
};

}  // namespace cskv
