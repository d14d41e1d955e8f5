// Host-only check of the call-slot bookkeeping (pn_slots.hpp) with a fake
// runtime: streams are integers, an event remembers the stream and the
// sequence number of its last record, and every wait, launch and record is
// logged.  Prints "ok" or the first failed check and exits nonzero.
#include <cstdio>
#include <thread>
#include <vector>

#include "pn_slots.hpp"

namespace {

struct Log {
    int kind;      // 0 wait, 1 launch, 2 record
    int stream, slot, event_seq;
};

struct FakeOps {
    using Stream = int;
    struct Ev {
        int id = -1, stream = -1, seq = -1;
    };
    using Event = Ev*;
    bool capture = false;
    int next_id = 0, created = 0, destroyed = 0, seq = 0;
    std::vector<Log> log;
    Ev pool[4096];
    int capturing(Stream, bool* c) { *c = capture; return 0; }
    int create(Event* e) { *e = &pool[next_id++]; (*e)->id = next_id - 1; ++created; return 0; }
    int wait(Stream s, Event e) { log.push_back({0, s, -1, e->seq}); return 0; }
    int record(Event e, Stream s) {
        e->stream = s; e->seq = seq - 1; log.push_back({2, s, -1, e->seq}); return 0;
    }
    int destroy(Event) { ++destroyed; return 0; }
    int launch(Stream s, int slot) { log.push_back({1, s, slot, seq}); ++seq; return 0; }
};

int fails = 0;
void check(bool c, const char* what) {
    if (!c && fails++ == 0) std::printf("FAILED: %s\n", what);
}

}  // namespace

int main() {
    using T = pn::SlotTable<FakeOps, 4, 3>;
    // 1. ring slots in turn; the first use of a slot waits for nothing, a
    //    reuse waits for the event recorded after the launch that used it last
    {
        static T t;
        FakeOps ops;
        std::vector<int> slots;
        for (int i = 0; i < 10; ++i) {
            const int s = i % 2;     // two streams
            check(t.run(ops, s, -5, [&](int k) { slots.push_back(k); return ops.launch(s, k); }) == 0, "run ok");
        }
        for (int i = 0; i < 10; ++i) check(slots[i] == i % 4, "ring order");
        check(ops.created == 4, "one event per ring slot");
        // per launch i: [wait] launch record
        int launches = 0, waits = 0;
        for (size_t j = 0; j < ops.log.size(); ++j) {
            const Log& L = ops.log[j];
            if (L.kind == 1) {
                const int i = L.event_seq;   // launch sequence number
                const bool reuse = i >= 4;
                if (reuse) {
                    check(j > 0 && ops.log[j - 1].kind == 0, "reuse is preceded by a wait");
                    check(ops.log[j - 1].event_seq == i - 4, "the wait is on the slot's previous launch");
                    check(ops.log[j - 1].stream == L.stream, "the wait is on the new call's stream");
                } else {
                    check(j == 0 || ops.log[j - 1].kind != 0, "first use waits for nothing");
                }
                check(j + 1 < ops.log.size() && ops.log[j + 1].kind == 2 && ops.log[j + 1].event_seq == i &&
                          ops.log[j + 1].stream == L.stream,
                      "each launch is followed by a record on its stream");
                ++launches;
            } else if (L.kind == 0) {
                ++waits;
            }
        }
        check(launches == 10 && waits == 6, "launch and wait counts");
        // 2. captured calls take slots of their own, never a ring slot, no events
        ops.capture = true;
        const size_t before = ops.log.size();
        std::vector<int> cs;
        for (int i = 0; i < 3; ++i)
            check(t.run(ops, 0, -5, [&](int k) { cs.push_back(k); return ops.launch(0, k); }) == 0, "capture ok");
        check(cs.size() == 3 && cs[0] == 4 && cs[1] == 5 && cs[2] == 6, "capture slots after the ring");
        for (size_t j = before; j < ops.log.size(); ++j) check(ops.log[j].kind == 1, "no event use under capture");
        bool called = false;
        check(t.run(ops, 0, -5, [&](int) { called = true; return 0; }) == -5, "capture pool exhausted");
        check(!called, "nothing launched when the pool is exhausted");
        check(t.captured_slots_used() == 3, "pool count");
        // 3. the ring continues where it was, unaffected by the captures
        ops.capture = false;
        int k2 = -1;
        check(t.run(ops, 1, -5, [&](int k) { k2 = k; return ops.launch(1, k); }) == 0, "run after capture");
        check(k2 == 10 % 4, "ring position kept");
        // 4. a failed launch records nothing; the slot's previous event stays the one to wait for
        int kf = -1;
        check(t.run(ops, 0, -5, [&](int k) { kf = k; return -3; }) == -3, "launch error passed through");
        const int seq_before = ops.seq;
        for (int i = 0; i < 3; ++i) t.run(ops, 0, -5, [&](int k) { return ops.launch(0, k); });
        int k4 = -1;
        const size_t at = ops.log.size();
        check(t.run(ops, 0, -5, [&](int k) { k4 = k; return ops.launch(0, k); }) == 0 && k4 == kf, "wrap to failed slot");
        check(ops.log[at].kind == 0 && ops.log[at].event_seq < seq_before, "waits on the last successful launch");
        // 5. reset destroys the events and empties both pools
        check(t.reset(ops) == 0 && ops.destroyed == 4, "reset destroys events");
        int k5 = -1;
        check(t.run(ops, 0, -5, [&](int k) { k5 = k; return ops.launch(0, k); }) == 0 && k5 == 0, "ring restarts");
        ops.capture = true;
        int k6 = -1;
        check(t.run(ops, 0, -5, [&](int k) { k6 = k; return ops.launch(0, k); }) == 0 && k6 == 4, "capture pool refilled");
    }
    // 6. host threads: every run on a slot is bracketed by the slot's lock,
    //    so no two launches of one slot overlap even under contention
    {
        static std::mutex m;
        static int inside[8] = {};
        static int bad = 0, created = 0;
        struct SafeOps {
            using Stream = int;
            using Event = int;
            int capturing(Stream, bool* c) { *c = false; return 0; }
            int create(Event* e) { std::lock_guard<std::mutex> g(m); *e = created++; return 0; }
            int wait(Stream, Event) { return 0; }
            int record(Event, Stream) { return 0; }
            int destroy(Event) { return 0; }
        };
        static pn::SlotTable<SafeOps, 8, 1> ts;
        std::vector<std::thread> th;
        for (int w = 0; w < 8; ++w) {
            th.emplace_back([w]() {
                SafeOps ops;
                for (int i = 0; i < 2000; ++i) {
                    ts.run(ops, w, -5, [&](int k) {
                        { std::lock_guard<std::mutex> g(m); if (inside[k]++ != 0) ++bad; }
                        std::this_thread::yield();
                        { std::lock_guard<std::mutex> g(m); --inside[k]; }
                        return 0;
                    });
                }
            });
        }
        for (auto& x : th) x.join();
        check(bad == 0, "one launch at a time per slot across threads");
        check(created == 8, "one event per slot across threads");
    }
    if (fails == 0) std::printf("ok\n");
    return fails == 0 ? 0 : 1;
}
