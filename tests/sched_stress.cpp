// Multi-threaded stress of the serving scheduler core (sched.h) on the CPU
// fake backend.  Built and run by tests/test_sched_sanitizers.py under
// ThreadSanitizer and under AddressSanitizer + UndefinedBehaviorSanitizer.
// Exit code 0 when every invariant held.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../paper_1407_2089_amd/csrc/sched.h"

using namespace vr;

static std::atomic<int> g_errors{0};
static std::atomic<uint64_t> g_budget{uint64_t(1) << 30};

#define CHECK(cond)                                                             \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            g_errors.fetch_add(1);                                              \
        }                                                                       \
    } while (0)

int main() {
    std::atomic<int> refs{0};
    const int kFail = 13;
    {
        Scheduler sched(new FakeBackend(3, 50.0, kFail), 8, [] { return g_budget.load(); });
        const int clients = 4, per_client = 400;
        std::vector<std::thread> th;
        for (int c = 0; c < clients; ++c) {
            th.emplace_back([&, c] {
                std::mt19937 rng(1234 + c);
                std::vector<std::pair<uint64_t, int>> mine;
                for (int q = 0; q < per_client; ++q) {
                    auto job = std::make_unique<Job>();
                    const int w = (rng() % 11 == 0) ? kFail : 1 + (int)(rng() % 200);
                    const int h = 1 + (int)(rng() % 100);
                    job->params.width = w;
                    job->params.height = h;
                    job->refs = &refs;
                    job->info.rays = (uint64_t)w * h * 2;
                    // now and then a request larger than any budget
                    job->out_bytes = (rng() % 97 == 0) ? (uint64_t(1) << 40) : job->info.rays * 16;
                    uint64_t t = 0;
                    vr_status st = sched.submit(std::move(job), &t);
                    CHECK(st == VR_OK || st == VR_ERR_BUSY);
                    if (st == VR_OK) mine.push_back({t, w});
                    if (q % 50 == 0) std::this_thread::yield();
                }
                for (auto& m : mine) {
                    vr_ticket_info info{};
                    bool released = false;
                    for (;;) {
                        CHECK(sched.poll(m.first, &info) == VR_OK);
                        if (info.state >= 2) break;
                        // releasing an unfinished ticket is refused; the job
                        // may finish between the two calls, then it succeeds
                        const vr_status r = sched.release(m.first);
                        CHECK(r == VR_ERR_BUSY || r == VR_OK);
                        if (r == VR_OK) {
                            released = true;
                            break;
                        }
                        std::this_thread::yield();
                    }
                    if (released) {
                        CHECK(sched.poll(m.first, &info) == VR_ERR_NOT_FOUND);
                        continue;
                    }
                    CHECK(info.t_arrive_ns > 0 && info.t_done_ns >= info.t_arrive_ns);
                    if (info.state == 2) {
                        CHECK(info.err == VR_OK && m.second != kFail);
                        CHECK(info.t_arrive_ns <= info.t_admit_ns);
                        CHECK(info.t_admit_ns <= info.t_start_ns);
                        CHECK(info.t_start_ns <= info.t_done_ns);
                    } else {
                        CHECK(info.err == VR_ERR_DEVICE || info.err == VR_ERR_OUT_OF_MEMORY);
                    }
                    CHECK(sched.release(m.first) == VR_OK);
                    CHECK(sched.poll(m.first, &info) == VR_ERR_NOT_FOUND);
                }
            });
        }
        // The budget moves while requests flow (volumes created and destroyed).
        std::thread budget([&] {
            for (int k = 0; k < 200; ++k) {
                g_budget.store(k % 2 ? (uint64_t(1) << 22) : (uint64_t(1) << 30));
                std::this_thread::sleep_for(std::chrono::microseconds(200));
            }
            g_budget.store(uint64_t(1) << 30);
        });
        // Someone polls unknown tickets and asks whether the loop is idle.
        std::thread prober([&] {
            vr_ticket_info info{};
            for (int k = 0; k < 2000; ++k) {
                CHECK(sched.poll(uint64_t(1) << 50, &info) == VR_ERR_NOT_FOUND);
                (void)sched.idle();
            }
        });
        for (auto& t : th) t.join();
        budget.join();
        prober.join();
        for (int k = 0; k < 1000 && !sched.idle(); ++k)
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        CHECK(sched.idle());
    }
    CHECK(refs.load() == 0);
    std::printf("errors %d\n", g_errors.load());
    return g_errors.load() == 0 ? 0 : 1;
}
