// Host-side test of the serving runtime (server.cpp) over the fake device of
// fake_device.cpp: the real scheduler and completion threads, the camera
// threads' submits and a polling thread, run under the thread sanitizer (and
// separately under the address and undefined-behaviour sanitizers).
// TEST INFRASTRUCTURE ONLY.
//
// Checked: every image a stream publishes equals the window definition
// (I/Q = the sums of (S0 - S2, S1 - S3) over the last min(c + 1, M) cycles
// since the last reset, re-summed here from the stored frames; amp = R), in
// camera-cycle order, alone and in a mix of three streams of different sizes;
// a held server launches nothing and then takes the three streams' cycles in
// one launch; submits while held and staging is full return QLD_E_AGAIN and
// take nothing; admission by budget in FIFO order; a frame-index gap resets
// the window; whole-cycle submits from three threads share launches; frames
// in page-locked memory take the direct copy.
// Exit status 0 on success; messages name the failed check.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/qld.h"

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                        \
    do {                                                        \
        if (!(cond)) {                                          \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                  \
            std::fprintf(stderr, "\n");                         \
            ++g_fail;                                           \
        }                                                       \
    } while (0)

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Cam {
    int H, W, M;
    std::vector<std::vector<uint16_t>> cycles;   // [cycle][4 * H * W]
};

Cam make_cam(int H, int W, int M, int n, unsigned seed) {
    Cam c{H, W, M, {}};
    std::mt19937 rng(seed);
    std::uniform_int_distribution<int> u(0, 4095);
    for (int k = 0; k < n; ++k) {
        std::vector<uint16_t> f(4 * (size_t)H * W);
        for (auto &v : f) v = (uint16_t)u(rng);
        c.cycles.push_back(std::move(f));
    }
    return c;
}

qld_frame_desc desc(int H, int W) {
    qld_frame_desc d{};
    d.H = H;
    d.W = W;
    d.row_pitch = W;
    d.frame_stride = (int64_t)H * W;
    d.dtype = QLD_U16;
    d.bits = 12;
    return d;
}

// R of the window after camera cycle k, whose window began at cycle k0.
std::vector<float> expected_amp(const Cam &c, int k0, int k) {
    const size_t px = (size_t)c.H * c.W;
    std::vector<float> a(px);
    const int first = std::max(k0, k - c.M + 1);
    for (size_t p = 0; p < px; ++p) {
        int64_t I = 0, Q = 0;
        for (int j = first; j <= k; ++j) {
            const uint16_t *f = c.cycles[j].data();
            I += (int64_t)f[p] - f[2 * px + p];
            Q += (int64_t)f[px + p] - f[3 * px + p];
        }
        a[p] = (float)std::sqrt((double)(uint64_t)(I * I + Q * Q));
    }
    return a;
}

struct Got {
    int64_t cycle;
    int warm;
    int64_t seq;
    std::vector<float> amp;
};

// Polls until stop is set and nothing is left; copies every image at once.
struct Poller {
    qld_server *s;
    std::atomic<bool> stop{false};
    std::mutex mu;
    std::map<int, std::vector<Got>> got;
    std::thread th;

    explicit Poller(qld_server *srv) : s(srv) {
        th = std::thread([this] {
            qld_result r[64];
            while (true) {
                int32_t n = 0;
                CHECK(qld_stream_poll(s, r, 64, &n) == QLD_OK, "poll");
                for (int i = 0; i < n; ++i) {
                    Got g{r[i].cycle, r[i].warm, r[i].seq,
                          std::vector<float>(r[i].amp, r[i].amp + (size_t)r[i].H * r[i].W)};
                    int32_t valid = 0;
                    CHECK(qld_stream_result_valid(s, &r[i], &valid) == QLD_OK && valid == 1,
                          "result of stream %d cycle %lld overwritten before it was copied", r[i].stream_id,
                          (long long)r[i].cycle);
                    std::lock_guard<std::mutex> lk(mu);
                    got[r[i].stream_id].push_back(std::move(g));
                }
                if (n == 0) {
                    if (stop.load()) break;
                    std::this_thread::sleep_for(std::chrono::microseconds(200));
                }
            }
        });
    }
    void finish() {
        stop.store(true);
        th.join();
    }
};

void check_stream(const char *what, const Cam &cam, const std::vector<Got> &g, int n_cycles, int reset_at = -1) {
    CHECK((int)g.size() == n_cycles, "%s: %zu images for %d cycles", what, g.size(), n_cycles);
    for (size_t i = 0; i < g.size() && i < (size_t)n_cycles; ++i) {
        const int k = (int)g[i].cycle;
        CHECK(k == (int)i + (reset_at >= 0 && (int)i >= reset_at ? 1 : 0), "%s: image %zu has cycle %d", what, i, k);
        const int k0 = reset_at >= 0 && k > reset_at ? reset_at + 1 : 0;
        const int wc = k - k0;                      // window cycle
        CHECK(g[i].warm == (wc + 1 >= cam.M ? 1 : 0), "%s: cycle %d warm %d", what, k, g[i].warm);
        CHECK(i == 0 || g[i].seq > g[i - 1].seq, "%s: seq not increasing at cycle %d", what, k);
        const std::vector<float> e = expected_amp(cam, k0, k);
        CHECK(e == g[i].amp, "%s: image of cycle %d differs from the window definition", what, k);
    }
}

// Three streams of different sizes, fed frame by frame by one thread each.
std::vector<std::vector<Got>> run_mix(const std::vector<Cam> &cams, const std::vector<int> &which, int n) {
    qld_server *s = nullptr;
    CHECK(qld_server_create((size_t)1 << 30, 64, 0, &s) == QLD_OK, "create");
    std::vector<int32_t> ids(which.size());
    for (size_t i = 0; i < which.size(); ++i) {
        const Cam &c = cams[which[i]];
        const qld_frame_desc d = desc(c.H, c.W);
        CHECK(qld_stream_open(s, &d, c.M, 0, QLD_MODE_PLAIN, &ids[i]) == QLD_OK, "open");
    }
    Poller poll(s);
    std::vector<std::thread> th;
    for (size_t i = 0; i < which.size(); ++i)
        th.emplace_back([&, i] {
            const Cam &c = cams[which[i]];
            const size_t px = (size_t)c.H * c.W;
            for (int k = 0; k < n; ++k)
                for (int f = 0; f < 4; ++f)
                    CHECK(qld_stream_submit(s, ids[i], c.cycles[k].data() + f * px, 4 * k + f, now_ns()) == QLD_OK,
                          "submit");
        });
    for (auto &t : th) t.join();
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    poll.finish();
    std::vector<std::vector<Got>> out;
    for (size_t i = 0; i < which.size(); ++i) out.push_back(poll.got[ids[i]]);
    CHECK(qld_server_destroy(s) == QLD_OK, "destroy");
    return out;
}

void test_mix_equals_alone(const std::vector<Cam> &cams) {
    const int n = 24;
    auto mix = run_mix(cams, {0, 1, 2}, n);
    for (int i = 0; i < 3; ++i) {
        auto alone = run_mix(cams, {i}, n);
        check_stream("mix", cams[i], mix[i], n);
        check_stream("alone", cams[i], alone[0], n);
        CHECK(alone[0].size() == mix[i].size(), "alone/mix sizes");
        for (size_t k = 0; k < alone[0].size() && k < mix[i].size(); ++k)
            CHECK(alone[0][k].amp == mix[i][k].amp, "stream %d cycle %zu: alone and mix differ", i, k);
    }
}

void test_hold_one_launch(const std::vector<Cam> &cams) {
    qld_server *s = nullptr;
    CHECK(qld_server_create((size_t)1 << 30, 16, 0, &s) == QLD_OK, "create");
    int32_t ids[3];
    for (int i = 0; i < 3; ++i) {
        const qld_frame_desc d = desc(cams[i].H, cams[i].W);
        CHECK(qld_stream_open(s, &d, cams[i].M, 0, QLD_MODE_PLAIN, &ids[i]) == QLD_OK, "open");
    }
    CHECK(qld_server_hold(s, 1) == QLD_OK, "hold");
    for (int i = 0; i < 3; ++i)
        CHECK(qld_stream_submit_cycle(s, ids[i], cams[i].cycles[0].data(), 0, now_ns()) == QLD_OK, "submit_cycle");
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    qld_result r[8];
    int32_t n = -1;
    CHECK(qld_stream_poll(s, r, 8, &n) == QLD_OK && n == 0, "a held server published %d images", n);
    int64_t b = 0, c = 0;
    int32_t mx = 0;
    size_t used = 0;
    CHECK(qld_server_stats(s, &b, &c, &mx, &used) == QLD_OK && b == 0, "a held server launched %lld", (long long)b);
    // Staging holds 4 cycles per stream: while held, the fifth waits for
    // nothing and is refused without being taken.
    for (int k = 1; k < 4; ++k)
        CHECK(qld_stream_submit_cycle(s, ids[0], cams[0].cycles[k].data(), 4 * k, now_ns()) == QLD_OK, "fill");
    CHECK(qld_stream_submit_cycle(s, ids[0], cams[0].cycles[4].data(), 16, now_ns()) == QLD_E_AGAIN,
          "fifth held cycle not refused");
    CHECK(qld_server_hold(s, 0) == QLD_OK, "release");
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    CHECK(qld_server_stats(s, &b, &c, &mx, &used) == QLD_OK, "stats");
    CHECK(mx == 3, "held cycles of three streams took %d streams per launch at most", mx);
    CHECK(c == 6, "%lld cycles processed, 6 submitted", (long long)c);
    // The refused cycle can be submitted now.
    CHECK(qld_stream_submit_cycle(s, ids[0], cams[0].cycles[4].data(), 16, now_ns()) == QLD_OK, "resubmit");
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    std::vector<Got> g;
    while (true) {
        CHECK(qld_stream_poll(s, r, 8, &n) == QLD_OK, "poll");
        if (n == 0) break;
        for (int i = 0; i < n; ++i)
            if (r[i].stream_id == ids[0])
                g.push_back(Got{r[i].cycle, r[i].warm, r[i].seq,
                                std::vector<float>(r[i].amp, r[i].amp + (size_t)r[i].H * r[i].W)});
    }
    check_stream("held", cams[0], g, 5);
    CHECK(qld_server_destroy(s) == QLD_OK, "destroy");
}

void test_admission_and_gap(const std::vector<Cam> &cams) {
    qld_server *probe = nullptr;
    CHECK(qld_server_create((size_t)1 << 30, 8, 0, &probe) == QLD_OK, "create");
    size_t need[3];
    for (int i = 0; i < 3; ++i) {
        const qld_frame_desc d = desc(cams[i].H, cams[i].W);
        need[i] = qld_server_stream_bytes(probe, &d, cams[i].M, 0, QLD_MODE_PLAIN);
        CHECK(need[i] > 0, "stream bytes");
    }
    CHECK(qld_server_destroy(probe) == QLD_OK, "destroy");
    qld_server *s = nullptr;
    CHECK(qld_server_create(need[0] + need[1], 8, 0, &s) == QLD_OK, "create");
    int32_t ids[3];
    qld_status st[3];
    for (int i = 0; i < 3; ++i) {
        const qld_frame_desc d = desc(cams[i].H, cams[i].W);
        st[i] = qld_stream_open(s, &d, cams[i].M, 0, QLD_MODE_PLAIN, &ids[i]);
    }
    CHECK(st[0] == QLD_OK && st[1] == QLD_OK && st[2] == QLD_E_AGAIN, "admission %d %d %d", st[0], st[1], st[2]);
    int32_t state = 0;
    CHECK(qld_stream_state(s, ids[2], &state) == QLD_OK && state == QLD_STREAM_PENDING, "pending state");
    CHECK(qld_stream_submit(s, ids[2], cams[2].cycles[0].data(), 0, now_ns()) == QLD_E_AGAIN, "submit to pending");
    CHECK(qld_stream_close(s, ids[0]) == QLD_OK, "close");
    CHECK(qld_stream_state(s, ids[2], &state) == QLD_OK && state == QLD_STREAM_ACTIVE, "admitted after close");
    // Gap: cycles 0..2, then cycle 4 (cycle 3 lost): the window restarts at 4.
    const Cam &c = cams[2];
    const size_t px = (size_t)c.H * c.W;
    Poller poll(s);
    for (int k = 0; k < 8; ++k) {
        if (k == 3) continue;
        for (int f = 0; f < 4; ++f) {
            const qld_status r = qld_stream_submit(s, ids[2], c.cycles[k].data() + f * px, 4 * k + f, now_ns());
            CHECK(r == (k == 4 && f == 0 ? QLD_E_GAP : QLD_OK), "submit cycle %d frame %d: %d", k, f, r);
        }
    }
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    poll.finish();
    check_stream("gap", c, poll.got[ids[2]], 7, 3);
    CHECK(qld_server_destroy(s) == QLD_OK, "destroy");
}

void test_flood(const std::vector<Cam> &cams) {
    qld_server *s = nullptr;
    CHECK(qld_server_create((size_t)1 << 30, 8, 0, &s) == QLD_OK, "create");
    int32_t ids[3];
    for (int i = 0; i < 3; ++i) {
        const qld_frame_desc d = desc(cams[i].H, cams[i].W);
        CHECK(qld_stream_open(s, &d, cams[i].M, 0, QLD_MODE_PLAIN, &ids[i]) == QLD_OK, "open");
    }
    const int n = 60;
    std::atomic<int> polled{0};
    std::atomic<bool> stop{false};
    std::thread pt([&] {          // metadata only: the slots are reused under it
        qld_result r[64];
        while (true) {
            int32_t k = 0;
            CHECK(qld_stream_poll(s, r, 64, &k) == QLD_OK, "poll");
            polled += k;
            if (k == 0) {
                if (stop.load()) break;
                std::this_thread::sleep_for(std::chrono::microseconds(100));
            }
        }
    });
    std::vector<std::thread> th;
    for (int i = 0; i < 3; ++i)
        th.emplace_back([&, i] {
            for (int k = 0; k < n; ++k)
                CHECK(qld_stream_submit_cycle(s, ids[i], cams[i].cycles[k % cams[i].cycles.size()].data(), 4 * k,
                                              now_ns()) == QLD_OK,
                      "submit_cycle");
        });
    for (auto &t : th) t.join();
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    stop.store(true);
    pt.join();
    int64_t b = 0, c = 0;
    int32_t mx = 0;
    size_t used = 0;
    CHECK(qld_server_stats(s, &b, &c, &mx, &used) == QLD_OK, "stats");
    CHECK(c == 3 * n && polled.load() == 3 * n, "cycles %lld polled %d of %d", (long long)c, polled.load(), 3 * n);
    CHECK(b <= c && b > 0, "launches %lld for %lld cycles", (long long)b, (long long)c);
    std::printf("flood: %lld cycles in %lld launches, up to %d streams per launch\n", (long long)c, (long long)b, mx);
    CHECK(qld_server_destroy(s) == QLD_OK, "destroy");
}

// Frames in page-locked memory are copied straight from the caller's buffer;
// the call returns once that copy is done, so the buffer may be refilled at once.
void test_pinned_submit(const std::vector<Cam> &cams) {
    const Cam &c = cams[1];
    const size_t bytes = 4 * (size_t)c.H * c.W * sizeof(uint16_t);
    void *pin = nullptr;
    CHECK(hipHostMalloc(&pin, bytes, hipHostMallocDefault) == hipSuccess, "page-locked buffer");
    qld_server *s = nullptr;
    CHECK(qld_server_create((size_t)1 << 30, 64, 0, &s) == QLD_OK, "create");
    int32_t id = 0;
    const qld_frame_desc d = desc(c.H, c.W);
    CHECK(qld_stream_open(s, &d, c.M, 0, QLD_MODE_PLAIN, &id) == QLD_OK, "open");
    Poller poll(s);
    const int n = 20;
    for (int k = 0; k < n; ++k) {
        std::memcpy(pin, c.cycles[k].data(), bytes);
        CHECK(qld_stream_submit_cycle(s, id, pin, 4 * k, now_ns()) == QLD_OK, "pinned submit_cycle");
    }
    // Per frame from page-locked memory too.
    const size_t fb = (size_t)c.H * c.W * sizeof(uint16_t);
    for (int k = n; k < n + 4; ++k)
        for (int f = 0; f < 4; ++f) {
            std::memcpy(pin, c.cycles[k].data() + f * (size_t)c.H * c.W, fb);
            CHECK(qld_stream_submit(s, id, pin, 4 * k + f, now_ns()) == QLD_OK, "pinned submit");
        }
    CHECK(qld_server_drain(s) == QLD_OK, "drain");
    poll.finish();
    check_stream("pinned", c, poll.got[id], n + 4);
    CHECK(qld_server_destroy(s) == QLD_OK, "destroy");
    CHECK(hipHostFree(pin) == hipSuccess, "free");
}

}  // namespace

int main() {
    std::vector<Cam> cams = {make_cam(8, 24, 4, 24, 1), make_cam(16, 40, 6, 24, 2), make_cam(5, 8, 3, 24, 3)};
    test_mix_equals_alone(cams);
    test_hold_one_launch(cams);
    test_admission_and_gap(cams);
    test_flood(cams);
    test_pinned_submit(cams);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("server host test: all checks passed\n");
    return 0;
}
