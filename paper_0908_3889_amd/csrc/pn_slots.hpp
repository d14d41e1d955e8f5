// pn_slots.hpp -- bookkeeping of the call slots of persistent launches.
//
// A persistent launch needs device memory of its own while it runs: a work
// counter that its waves claim inspirals from, and the launch descriptor its
// refill passes read.  Each launch takes one fixed-size slot of a per-device
// table; a slot must not be rewritten while a launch that uses it may still
// run, or that launch would claim from a reset counter and write through
// another call's pointers, silently (Sec. III: kernel failures on the GPU
// go unreported unless checked for).
//
// Direct calls take the slots of a ring in turn.  After each launch an event
// is recorded on its stream in the slot; before a slot is reused, the new
// call's stream waits for that event, so a slot is never rewritten while the
// launch that used it can run, whatever streams the two calls are on.  A
// per-slot lock makes the wait / launch / record sequence atomic with respect
// to other host threads.
//
// A call made while its stream is being captured into a graph takes a slot
// of its own from a second pool, never reused until the context is released:
// every replay of the graph zeroes the counter and rewrites the descriptor of
// that slot, so it must not be shared with later calls, and no event can be
// recorded or waited for across the capture.  Replays of one graph must not
// overlap one another (they also write the same outputs).  When that pool is
// used up the call fails with a distinct code and launches nothing.
//
// The logic is templated on the runtime operations so that it can be
// exercised on the host without a device.
#pragma once

#include <atomic>
#include <mutex>

namespace pn {

template <class Ops, int RING, int CAPTURE>
class SlotTable {
   public:
    using Stream = typename Ops::Stream;
    using Event = typename Ops::Event;
    static constexpr int kRing = RING;
    static constexpr int kCapture = CAPTURE;

    // Calls launch(slot) with the index of a slot that no running launch
    // uses (ring slots 0 .. RING-1, capture slots RING .. RING+CAPTURE-1).
    // Returns 0, launch's nonzero result, an Ops error, or exhausted_code
    // when a capture needs a slot and none is left.
    template <class F>
    int run(Ops& ops, Stream s, int exhausted_code, F&& launch) {
        bool cap = false;
        if (int e = ops.capturing(s, &cap)) return e;
        if (cap) {
            int k = next_capture_.load(std::memory_order_relaxed);
            do {
                if (k >= CAPTURE) return exhausted_code;
            } while (!next_capture_.compare_exchange_weak(k, k + 1, std::memory_order_relaxed));
            return launch(RING + k);
        }
        const int k = (int)(next_.fetch_add(1, std::memory_order_relaxed) % (unsigned)RING);
        std::lock_guard<std::mutex> lk(mu_[k]);
        if (!have_event_[k]) {
            if (int e = ops.create(&ev_[k])) return e;
            have_event_[k] = true;
        }
        if (recorded_[k]) {
            if (int e = ops.wait(s, ev_[k])) return e;
        }
        if (int e = launch(k)) return e;
        if (int e = ops.record(ev_[k], s)) {
            recorded_[k] = false;      // the launch is queued but not tracked: nothing to wait for
            return e;
        }
        recorded_[k] = true;
        return 0;
    }

    // Destroys the events and empties both pools (the caller guarantees that
    // nothing of the library is queued or running on the device).
    int reset(Ops& ops) {
        int rc = 0;
        for (int k = 0; k < RING; ++k) {
            std::lock_guard<std::mutex> lk(mu_[k]);
            if (have_event_[k]) {
                if (int e = ops.destroy(ev_[k])) rc = e;
                have_event_[k] = false;
            }
            recorded_[k] = false;
        }
        next_.store(0, std::memory_order_relaxed);
        next_capture_.store(0, std::memory_order_relaxed);
        return rc;
    }

    int captured_slots_used() const { return next_capture_.load(std::memory_order_relaxed); }

   private:
    std::atomic<unsigned> next_{0};
    std::atomic<int> next_capture_{0};
    std::mutex mu_[RING];
    Event ev_[RING] = {};
    bool have_event_[RING] = {};
    bool recorded_[RING] = {};
};

}  // namespace pn
