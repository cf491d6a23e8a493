// Serving runtime: many camera streams on one GPU with continuous batching.
//
// The paper's real-time loop (Supplementary, "Timing sequence for hybrid
// parallelisation") runs one thread that prepares frames, one that feeds the
// GPU and one kernel per frame, coordinated by status flags.  Here the same
// roles are played by
//   * the caller's camera threads (qld_stream_submit): copy a frame into
//     pinned staging and enqueue its host-to-device copy on the copy stream;
//   * a scheduler thread: takes every ready cycle of every admitted stream
//     and applies them in ONE launch of the batched window kernel (streams of
//     different sizes share the launch), after waiting on the copy events;
//   * a completion thread: waits for each launch's event, stamps the host
//     time and publishes the images (qld_stream_poll).
// HIP stream order and events replace the flags.  Streams are admitted while
// the sum of their device footprints fits the HBM budget; the rest wait in
// FIFO order and are admitted as closes free memory.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "window.hpp"

namespace qld {
namespace {

constexpr int kStageCycles = 4;      // staged cycles per stream on the device
constexpr int kPinnedFrames = 8;     // pinned host frame buffers per stream
constexpr int kMaxCyclesPerJob = 8;  // cycles of one stream applied per launch

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct StreamRec {
    int id = 0;
    int state = QLD_STREAM_PENDING;
    qld_frame_desc d{};
    int eb = 2;
    int M = 1, Ms = 0, mode = 0;
    size_t bytes = 0;

    qld_window *win = nullptr;
    uint8_t *stage = nullptr;       // [kStageCycles][4][H][Wp] samples
    int64_t rp_b = 0, fs_b = 0, slot_b = 0;
    float *out_amp = nullptr;       // [out_slots][H][W]
    int32_t *out_iq = nullptr;      // [out_slots][2 or 4][H][W] when the server keeps I/Q
    uint8_t *pin = nullptr;         // [kPinnedFrames][H][W]
    size_t frame_bytes = 0;
    hipEvent_t pin_ev[kPinnedFrames] = {};
    bool pin_used[kPinnedFrames] = {};
    int pin_next = 0;
    hipEvent_t slot_ev[kStageCycles] = {};
    uint64_t slot_tarr[kStageCycles] = {};
    int64_t slot_cam_cycle[kStageCycles] = {};
    bool slot_reset[kStageCycles] = {};

    int64_t next_frame = 0;     // expected next frame index
    int cur = 0;                // frames of the cycle being filled
    bool dropping = false;      // after a gap: drop frames until a cycle starts
    bool reset_next = true;     // next complete cycle starts a fresh window
    int64_t submitted = 0;      // complete cycles handed to the scheduler
    int64_t launched = 0;
    int64_t done = 0;
    int64_t win_c = 0;          // window cycle index of the next launched cycle
    std::deque<int64_t> ready;  // lifetime cycle numbers awaiting launch
};

struct CycleRef {
    StreamRec *s;
    int64_t k;          // lifetime cycle number
    int64_t cam_cycle;
    uint64_t t_arr;
    int warm;
    int out_slot;
};

struct Inflight {
    hipEvent_t ev;
    std::vector<CycleRef> cycles;
};

}  // namespace
}  // namespace qld

struct qld_server {
    size_t budget = 0;
    int out_slots = 4;
    int flags = 0;
    int device = 0;
    size_t in_use = 0;
    hipStream_t copy = nullptr, compute = nullptr;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_complete;
    std::map<int, std::unique_ptr<qld::StreamRec>> streams;
    std::deque<int> pending;  // FIFO of streams waiting for budget
    int next_id = 1;
    std::deque<qld_result> results;
    std::deque<qld::Inflight> inflight;
    std::vector<hipEvent_t> free_events;
    bool stop = false;
    std::thread sched, complete;
    int64_t batches = 0, cycles = 0;
    int32_t max_streams = 0;
    qld_status async_error = QLD_OK;
};

namespace qld {
namespace {

int padded_w(int W, int eb) { return (int)(ceil_div(W, window_vpx(eb)) * window_vpx(eb)); }

size_t stream_bytes(const qld_server *s, const qld_frame_desc *d, int M, int Ms) {
    int eb = 0;
    if (check_desc(d, &eb) != QLD_OK) return 0;
    const size_t wb = window_bytes(d, M, Ms);
    if (!wb && (size_t)d->H * d->W) return 0;
    const size_t npx = (size_t)d->H * d->W;
    const size_t stage = (size_t)kStageCycles * 4 * d->H * padded_w(d->W, eb) * eb;
    const size_t out = (size_t)s->out_slots * npx * 4;
    const size_t iq = (s->flags & 1) ? (size_t)s->out_slots * npx * 4 * (Ms > 0 ? 4 : 2) : 0;
    return wb + stage + out + iq;
}

void free_stream_mem(StreamRec *r) {
    if (r->win) qld_window_destroy(r->win);
    r->win = nullptr;
    if (r->stage) (void)hipFree(r->stage);
    if (r->out_amp) (void)hipFree(r->out_amp);
    if (r->out_iq) (void)hipFree(r->out_iq);
    if (r->pin) (void)hipHostFree(r->pin);
    r->stage = r->pin = nullptr;
    r->out_amp = nullptr;
    r->out_iq = nullptr;
    for (auto &e : r->pin_ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    for (auto &e : r->slot_ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
}

// Allocate the device/pinned memory of an admitted stream (mu held).
qld_status alloc_stream(qld_server *srv, StreamRec *r) {
    qld_status st = window_alloc(&r->d, r->M, r->Ms, &r->win);
    if (st != QLD_OK) return st;
    const int Wp = padded_w(r->d.W, r->eb);
    r->rp_b = (int64_t)Wp * r->eb;
    r->fs_b = r->rp_b * r->d.H;
    r->slot_b = 4 * r->fs_b;
    const size_t npx = (size_t)r->d.H * r->d.W;
    r->frame_bytes = npx * r->eb;
    hipError_t e = hipMalloc(&r->stage, (size_t)kStageCycles * r->slot_b + 16);
    if (e == hipSuccess) e = hipMemset(r->stage, 0, (size_t)kStageCycles * r->slot_b + 16);
    if (e == hipSuccess) e = hipMalloc(&r->out_amp, (size_t)srv->out_slots * npx * 4 + 16);
    if (e == hipSuccess && (srv->flags & 1))
        e = hipMalloc(&r->out_iq, (size_t)srv->out_slots * npx * 4 * (r->Ms > 0 ? 4 : 2) + 16);
    if (e == hipSuccess) e = hipHostMalloc(&r->pin, (size_t)kPinnedFrames * r->frame_bytes + 16, hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < kPinnedFrames; ++i)
        e = hipEventCreateWithFlags(&r->pin_ev[i], hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < kStageCycles; ++i)
        e = hipEventCreateWithFlags(&r->slot_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_stream_mem(r);
        set_error("stream allocation failed: %s", hipGetErrorString(e));
        return QLD_E_NOMEM;
    }
    return QLD_OK;
}

// Admit pending streams in FIFO order while they fit (mu held).
void admit_pending(qld_server *srv) {
    while (!srv->pending.empty()) {
        auto it = srv->streams.find(srv->pending.front());
        if (it == srv->streams.end()) {
            srv->pending.pop_front();
            continue;
        }
        StreamRec *r = it->second.get();
        if (srv->in_use + r->bytes > srv->budget) break;
        if (alloc_stream(srv, r) != QLD_OK) break;
        srv->in_use += r->bytes;
        r->state = QLD_STREAM_ACTIVE;
        srv->pending.pop_front();
    }
}

hipEvent_t take_event(qld_server *srv) {
    if (!srv->free_events.empty()) {
        hipEvent_t e = srv->free_events.back();
        srv->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void scheduler_loop(qld_server *srv) {
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    size_t rr = 0;  // round-robin start for fairness when a launch is full
    while (true) {
        srv->cv_sched.wait(lk, [&] {
            if (srv->stop) return true;
            for (auto &kv : srv->streams)
                if (!kv.second->ready.empty()) return true;
            return false;
        });
        std::vector<StreamRec *> order;
        for (auto &kv : srv->streams)
            if (!kv.second->ready.empty()) order.push_back(kv.second.get());
        if (order.empty()) {
            if (srv->stop) break;
            continue;
        }
        std::rotate(order.begin(), order.begin() + (rr % order.size()), order.end());
        ++rr;
        // Group by kernel variant (sample size, ring width); one launch per group.
        std::map<int, std::vector<StreamRec *>> groups;
        for (StreamRec *r : order) groups[r->eb * 2 + (r->d.bits > 15 ? 1 : 0)].push_back(r);

        for (auto &g : groups) {
            WinBatch b{};
            std::vector<CycleRef> refs;
            std::vector<hipEvent_t> waits;
            int tiles = 0;
            for (StreamRec *r : g.second) {
                if (b.n_jobs == kMaxJobs) break;
                WinJob &J = b.job[b.n_jobs];
                const int64_t k0 = r->ready.front();
                const int slot0 = (int)(k0 % kStageCycles);
                const bool fresh = r->slot_reset[slot0];
                int n = 0;
                while (n < (int)r->ready.size() && n < kMaxCyclesPerJob) {
                    const int64_t k = r->ready[n];
                    if (n > 0 && r->slot_reset[k % kStageCycles]) break;   // a reset starts its own job
                    ++n;
                }
                const int64_t c0 = fresh ? 0 : r->win_c;
                const int npx = r->d.H * r->d.W;
                J.stage = r->stage;
                J.rp_b = r->rp_b;
                J.fs_b = r->fs_b;
                J.slot_b = r->slot_b;
                J.n_stage = kStageCycles;
                J.stage0 = slot0;
                J.H = r->d.H;
                J.W = r->d.W;
                J.Wp = r->win->Wp;
                J.M = r->M;
                J.Ms = r->Ms;
                J.c0 = c0;
                J.n_cycles = n;
                J.fresh = fresh ? 1 : 0;
                J.ring = r->win->ring;
                J.I = r->win->I;
                J.Q = r->win->Q;
                J.Is = r->win->Is;
                J.Qs = r->win->Qs;
                J.amp = r->out_amp;
                if (r->out_iq) {
                    const int per = r->Ms > 0 ? 4 : 2;
                    // Slot layout: [out_slots][per][H][W]; the kernel indexes
                    // slot * npx, so each plane gets its own base and stride.
                    (void)per;
                    J.Io = r->out_iq;
                    J.Qo = r->out_iq + (size_t)srv->out_slots * npx;
                    if (r->Ms > 0) {
                        J.Iso = r->out_iq + 2 * (size_t)srv->out_slots * npx;
                        J.Qso = r->out_iq + 3 * (size_t)srv->out_slots * npx;
                    }
                }
                J.out_slots = srv->out_slots;
                J.out0 = (int32_t)(k0 % srv->out_slots);
                J.tiles = (int32_t)ceil_div((int64_t)r->d.H * (J.Wp / window_vpx(r->eb)), 256);
                b.tile_start[b.n_jobs] = tiles;
                tiles += J.tiles;
                b.n_jobs++;
                for (int i = 0; i < n; ++i) {
                    const int64_t k = r->ready.front();
                    r->ready.pop_front();
                    const int sl = (int)(k % kStageCycles);
                    waits.push_back(r->slot_ev[sl]);
                    const int64_t c = c0 + i;
                    refs.push_back(CycleRef{r, k, r->slot_cam_cycle[sl], r->slot_tarr[sl], c + 1 >= r->M ? 1 : 0,
                                            (int)(k % srv->out_slots)});
                }
                r->win_c = c0 + n;
                r->launched += n;
            }
            b.tile_start[b.n_jobs] = tiles;
            if (b.n_jobs == 0) continue;
            hipEvent_t ev = take_event(srv);
            const int eb = g.first / 2;
            const bool wide = g.first & 1;
            lk.unlock();
            hipError_t e = hipSuccess;
            for (hipEvent_t w : waits)
                if (e == hipSuccess) e = hipStreamWaitEvent(srv->compute, w, 0);
            // Staging rows are padded to 16-byte multiples: the vector path always applies.
            if (e == hipSuccess) e = launch_window_batch(b, eb, wide, true, srv->compute);
            if (e == hipSuccess && ev) e = hipEventRecord(ev, srv->compute);
            lk.lock();
            if (e != hipSuccess || !ev) {
                srv->async_error = QLD_E_DEVICE;
                set_error("server launch failed: %s", hipGetErrorString(e));
            }
            srv->batches++;
            srv->max_streams = std::max<int32_t>(srv->max_streams, b.n_jobs);
            srv->inflight.push_back(Inflight{ev, std::move(refs)});
            srv->cv_complete.notify_one();
        }
    }
}

void completion_loop(qld_server *srv) {
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        srv->cv_complete.wait(lk, [&] { return srv->stop || !srv->inflight.empty(); });
        if (srv->inflight.empty()) {
            if (srv->stop) break;
            continue;
        }
        Inflight f = std::move(srv->inflight.front());
        srv->inflight.pop_front();
        lk.unlock();
        hipError_t e = f.ev ? hipEventSynchronize(f.ev) : hipErrorInvalidValue;
        const uint64_t t = now_ns();
        lk.lock();
        if (e != hipSuccess) {
            srv->async_error = QLD_E_DEVICE;
            set_error("server batch failed: %s", hipGetErrorString(e));
        }
        if (f.ev) srv->free_events.push_back(f.ev);
        for (const CycleRef &c : f.cycles) {
            StreamRec *r = c.s;
            qld_result res{};
            res.stream_id = r->id;
            res.warm = c.warm;
            res.cycle = c.cam_cycle;
            res.t_arrival_ns = c.t_arr;
            res.t_done_ns = t;
            res.amp = r->out_amp + (size_t)c.out_slot * r->d.H * r->d.W;
            res.H = r->d.H;
            res.W = r->d.W;
            srv->results.push_back(res);
            r->done++;
            srv->cycles++;
        }
        srv->cv_done.notify_all();
    }
}

StreamRec *find_stream(qld_server *s, int id) {
    auto it = s->streams.find(id);
    return it == s->streams.end() ? nullptr : it->second.get();
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_server_create(size_t hbm_budget_bytes, int32_t out_slots, int32_t flags,
                                        qld_server **out) {
    clear_error();
    if (!out || out_slots < 1 || out_slots > 1024) {
        set_error("out must be non-NULL and out_slots in 1..1024");
        return QLD_E_INVAL;
    }
    auto *s = new (std::nothrow) qld_server();
    if (!s) {
        set_error("host allocation failed");
        return QLD_E_NOMEM;
    }
    s->budget = hbm_budget_bytes;
    s->out_slots = out_slots;
    s->flags = flags;
    (void)hipGetDevice(&s->device);
    qld_status st = check_hip(hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking), "copy stream");
    if (st == QLD_OK) st = check_hip(hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking), "compute stream");
    if (st != QLD_OK) {
        if (s->copy) (void)hipStreamDestroy(s->copy);
        delete s;
        return st;
    }
    s->sched = std::thread(scheduler_loop, s);
    s->complete = std::thread(completion_loop, s);
    *out = s;
    return QLD_OK;
}

extern "C" size_t qld_server_stream_bytes(const qld_server *s, const qld_frame_desc *d, int32_t M_cycles,
                                          int32_t M_short) {
    if (!s) return 0;
    return stream_bytes(s, d, M_cycles, M_short);
}

extern "C" qld_status qld_stream_open(qld_server *s, const qld_frame_desc *d, int32_t M_cycles, int32_t M_short,
                                      int32_t mode, int32_t *stream_id) {
    clear_error();
    int eb = 0;
    if (!s || !stream_id) {
        set_error("server and stream_id must be non-NULL");
        return QLD_E_INVAL;
    }
    QLD_TRY(check_desc(d, &eb));
    if (d->H < 1 || d->W < 1) {
        set_error("a stream needs frames of at least 1x1 pixels");
        return QLD_E_SHAPE;
    }
    if (M_cycles < 1 || M_short < 0 || M_short > M_cycles || mode != QLD_MODE_PLAIN) {
        set_error("invalid window M=%d short=%d mode=%d", M_cycles, M_short, mode);
        return QLD_E_INVAL;
    }
    if ((uint64_t)M_cycles * ((1ull << d->bits) - 1) >= (1ull << 31)) {
        set_error("M=%d cycles of %d-bit data could overflow int32", M_cycles, d->bits);
        return QLD_E_OVERFLOW;
    }
    const size_t need = stream_bytes(s, d, M_cycles, M_short);
    if (need == 0 || need > s->budget) {
        set_error("stream needs %zu bytes, budget is %zu", need, s->budget);
        return QLD_E_BUDGET;
    }
    (void)hipSetDevice(s->device);
    std::lock_guard<std::mutex> lk(s->mu);
    auto r = std::make_unique<StreamRec>();
    r->id = s->next_id++;
    r->d = *d;
    r->d.row_pitch = d->W;
    r->d.frame_stride = (int64_t)d->H * d->W;
    r->eb = eb;
    r->M = M_cycles;
    r->Ms = M_short;
    r->mode = mode;
    r->bytes = need;
    StreamRec *rp = r.get();
    s->streams[r->id] = std::move(r);
    *stream_id = rp->id;
    if (s->pending.empty() && s->in_use + need <= s->budget) {
        qld_status st = alloc_stream(s, rp);
        if (st != QLD_OK) {
            s->streams.erase(rp->id);
            return st;
        }
        s->in_use += need;
        rp->state = QLD_STREAM_ACTIVE;
        return QLD_OK;
    }
    s->pending.push_back(rp->id);
    set_error("stream %d queued: %zu bytes needed, %zu of %zu in use", rp->id, need, s->in_use, s->budget);
    return QLD_E_AGAIN;
}

extern "C" qld_status qld_stream_state(qld_server *s, int32_t stream_id, int32_t *state) {
    clear_error();
    if (!s || !state) return QLD_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    StreamRec *r = find_stream(s, stream_id);
    *state = r ? r->state : QLD_STREAM_CLOSED;
    return QLD_OK;
}

extern "C" qld_status qld_stream_submit(qld_server *s, int32_t stream_id, const void *host_frame,
                                        int64_t frame_index, uint64_t t_arrival_ns) {
    clear_error();
    if (!s || !host_frame) {
        set_error("server and host_frame must be non-NULL");
        return QLD_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->async_error != QLD_OK) return s->async_error;
    StreamRec *r = find_stream(s, stream_id);
    if (!r || r->state == QLD_STREAM_CLOSED) {
        set_error("stream %d is not open", stream_id);
        return QLD_E_INVAL;
    }
    if (r->state == QLD_STREAM_PENDING) {
        set_error("stream %d is waiting for admission", stream_id);
        return QLD_E_AGAIN;
    }
    if (frame_index < r->next_frame) {
        set_error("frame index %lld < expected %lld", (long long)frame_index, (long long)r->next_frame);
        return QLD_E_INVAL;
    }
    qld_status ret = QLD_OK;
    if (frame_index > r->next_frame) {
        // A gap loses the phase alignment: drop the partial cycle, restart the window.
        r->cur = 0;
        r->dropping = true;
        r->reset_next = true;
        ret = QLD_E_GAP;
        set_error("frame index jumped from %lld to %lld: window reset", (long long)r->next_frame,
                  (long long)frame_index);
    }
    r->next_frame = frame_index + 1;
    const int phase = (int)(frame_index & 3);
    if (r->dropping) {
        if (phase != 0) return ret;   // wait for the first frame of a cycle
        r->dropping = false;
    }
    if (phase != r->cur) {
        // Stream started mid-cycle (first frame index not a multiple of 4).
        r->cur = 0;
        if (phase != 0) return ret;
    }
    const int64_t k = r->submitted;
    const int slot = (int)(k % kStageCycles);
    if (phase == 0) {
        // Back-pressure: the staging slot must have been consumed.
        s->cv_done.wait(lk, [&] { return r->done > k - kStageCycles || s->async_error != QLD_OK; });
        if (s->async_error != QLD_OK) return s->async_error;
    }
    const int p = r->pin_next;
    r->pin_next = (r->pin_next + 1) % kPinnedFrames;
    const bool used = r->pin_used[p];
    r->pin_used[p] = true;
    hipEvent_t pev = r->pin_ev[p];
    uint8_t *pin = r->pin + (size_t)p * r->frame_bytes;
    uint8_t *dst = r->stage + (size_t)slot * r->slot_b + (size_t)phase * r->fs_b;
    lk.unlock();

    hipError_t e = hipSuccess;
    if (used) e = hipEventSynchronize(pev);   // the pinned buffer's previous copy is done
    if (e == hipSuccess) {
        memcpy(pin, host_frame, r->frame_bytes);
        e = hipMemcpy2DAsync(dst, (size_t)r->rp_b, pin, (size_t)r->d.W * r->eb, (size_t)r->d.W * r->eb,
                             (size_t)r->d.H, hipMemcpyHostToDevice, s->copy);
    }
    if (e == hipSuccess) e = hipEventRecord(pev, s->copy);
    if (e == hipSuccess && phase == 3) e = hipEventRecord(r->slot_ev[slot], s->copy);

    lk.lock();
    if (e != hipSuccess) {
        set_error("frame copy failed: %s", hipGetErrorString(e));
        return QLD_E_DEVICE;
    }
    r->cur = phase + 1;
    if (phase == 3) {
        r->slot_tarr[slot] = t_arrival_ns;
        r->slot_cam_cycle[slot] = frame_index >> 2;
        r->slot_reset[slot] = r->reset_next;
        r->reset_next = false;
        r->ready.push_back(k);
        r->submitted++;
        r->cur = 0;
        s->cv_sched.notify_one();
    }
    return ret;
}

extern "C" qld_status qld_stream_poll(qld_server *s, qld_result *out, int32_t max, int32_t *n_out) {
    clear_error();
    if (!s || !n_out || (max > 0 && !out)) return QLD_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->results.empty()) {
        out[n++] = s->results.front();
        s->results.pop_front();
    }
    *n_out = n;
    return s->async_error;
}

extern "C" qld_status qld_server_drain(qld_server *s) {
    clear_error();
    if (!s) return QLD_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        if (s->async_error != QLD_OK) return true;
        for (auto &kv : s->streams)
            if (kv.second->done < kv.second->submitted) return false;
        return true;
    });
    return s->async_error;
}

extern "C" qld_status qld_stream_close(qld_server *s, int32_t stream_id) {
    clear_error();
    if (!s) return QLD_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    StreamRec *r = find_stream(s, stream_id);
    if (!r) {
        set_error("stream %d is not open", stream_id);
        return QLD_E_INVAL;
    }
    if (r->state == QLD_STREAM_PENDING) {
        s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), stream_id), s->pending.end());
        s->streams.erase(stream_id);
        return QLD_OK;
    }
    r->state = QLD_STREAM_CLOSED;
    s->cv_done.wait(lk, [&] { return r->done >= r->submitted || s->async_error != QLD_OK; });
    // Results already published keep pointing at this stream's output slots:
    // drop them so nobody reads freed memory.
    s->results.erase(std::remove_if(s->results.begin(), s->results.end(),
                                     [&](const qld_result &q) { return q.stream_id == stream_id; }),
                     s->results.end());
    lk.unlock();
    (void)hipStreamSynchronize(s->copy);
    lk.lock();
    free_stream_mem(r);
    s->in_use -= r->bytes;
    s->streams.erase(stream_id);
    admit_pending(s);
    return QLD_OK;
}

extern "C" qld_status qld_server_destroy(qld_server *s) {
    clear_error();
    if (!s) return QLD_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] {
            if (s->async_error != QLD_OK) return true;
            for (auto &kv : s->streams)
                if (kv.second->done < kv.second->submitted) return false;
            return true;
        });
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_complete.notify_all();
    if (s->sched.joinable()) s->sched.join();
    if (s->complete.joinable()) s->complete.join();
    (void)hipStreamSynchronize(s->compute);
    (void)hipStreamSynchronize(s->copy);
    for (auto &kv : s->streams) free_stream_mem(kv.second.get());
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    for (auto &f : s->inflight)
        if (f.ev) (void)hipEventDestroy(f.ev);
    (void)hipStreamDestroy(s->compute);
    (void)hipStreamDestroy(s->copy);
    delete s;
    return QLD_OK;
}

extern "C" qld_status qld_server_stats(const qld_server *s, int64_t *batches, int64_t *cycles,
                                       int32_t *max_streams_in_batch, size_t *bytes_in_use) {
    if (!s) return QLD_E_INVAL;
    auto *m = const_cast<qld_server *>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    if (batches) *batches = s->batches;
    if (cycles) *cycles = s->cycles;
    if (max_streams_in_batch) *max_streams_in_batch = s->max_streams;
    if (bytes_in_use) *bytes_in_use = s->in_use;
    return QLD_OK;
}

extern "C" qld_status qld_stream_result_iq(qld_server *s, const qld_result *res, const int32_t **I,
                                           const int32_t **Q, const int32_t **Is, const int32_t **Qs) {
    clear_error();
    if (!s || !res) return QLD_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    StreamRec *r = find_stream(s, res->stream_id);
    if (!r || !r->out_iq) {
        set_error("stream %d keeps no I/Q outputs", res->stream_id);
        return QLD_E_STATE;
    }
    const size_t npx = (size_t)r->d.H * r->d.W;
    const size_t slot = (size_t)(res->amp - r->out_amp) / npx;
    const size_t plane = (size_t)s->out_slots * npx;
    if (I) *I = r->out_iq + slot * npx;
    if (Q) *Q = r->out_iq + plane + slot * npx;
    if (Is) *Is = r->Ms > 0 ? r->out_iq + 2 * plane + slot * npx : nullptr;
    if (Qs) *Qs = r->Ms > 0 ? r->out_iq + 3 * plane + slot * npx : nullptr;
    return QLD_OK;
}
