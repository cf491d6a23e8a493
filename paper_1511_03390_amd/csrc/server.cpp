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
//     different sizes share the launch), after waiting on the copy events.
//     At most max_inflight launch rounds are on the device at once (one by
//     default): cycles that land while a round runs are gathered into the
//     next one, so under load a launch carries the cycles of several
//     streams (continuous batching) instead of one launch per cycle;
//   * a completion thread: waits for each launch's event, stamps the host
//     time and publishes the images (qld_stream_poll).
// A LEARNED stream (not in the paper) also runs its denoiser on the short
// window after each cycle, on the same compute stream and before the launch's
// event, and serves either that image or the plain long-window amplitude as
// its gate decides.
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

#include "serve_learned.hpp"
#include "window.hpp"

namespace qld {
namespace {

constexpr int kStageCycles = 4;      // staged cycles per stream on the device
constexpr int kPinnedCycles = 2;     // pinned host cycle buffers (4 frames each) per stream
constexpr int kPinnedFrames = 4 * kPinnedCycles;
constexpr int kMaxCyclesPerJob = 8;  // cycles of one stream applied per launch
constexpr int kMaxInflight = 64;

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
    int32_t *out_iq = nullptr;      // I/Q output planes, each [out_slots][H][W]:
    int32_t *Io = nullptr, *Qo = nullptr;     //   long window (server keeps I/Q)
    int32_t *Iso = nullptr, *Qso = nullptr;   //   short window (keeps I/Q, or LEARNED)

    // LEARNED streams.
    qld_denoiser *dn = nullptr;
    float gate_thr = 0.05f;
    const float *dn_y = nullptr, *dn_gate = nullptr;   // the denoiser's output tensors
    float *served = nullptr;        // [out_slots][H][W] served images
    float *x = nullptr;             // [H][W][2] network input
    float *scale = nullptr;         // [1]
    uint64_t *sumS = nullptr;       // [1] short-window sample sum
    uint64_t *csum = nullptr;       // [ring][kCycleSumBlocks] per-cycle partial sums
    uint32_t *pcs = nullptr;        // [ring][H][W] per-pixel cycle sums
    uint32_t *psS = nullptr;        // [H][W] per-pixel short-window sums
    float *gate_dev = nullptr;      // [out_slots]
    float *gate_host = nullptr;     // pinned [out_slots]
    int ring = 0;
    uint8_t *pin = nullptr;         // [kPinnedCycles][4][H][W]: frame (k, phase) at k % kPinnedCycles
    size_t frame_bytes = 0;
    hipEvent_t pin_ev[kPinnedFrames] = {};   // last copy out of each pinned frame
    hipEvent_t direct_ev = nullptr;          // copy straight from a caller's page-locked frames
    hipStream_t copy = nullptr;              // this stream's host-to-device copies
    bool pin_used[kPinnedFrames] = {};
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
    float gate_thr;     // LEARNED: threshold the launch used
};

// The learned work of one job: cycles c0 .. c0+n-1 of a LEARNED stream.
struct LearnedJob {
    StreamRec *r;
    qld_denoiser *dn;
    const float *y, *gate;
    float thr;
    int64_t c0;
    int n, out0, stage0;
};

struct Inflight {
    hipEvent_t ev;
    std::vector<CycleRef> cycles;
    bool round_end;     // last launch of a scheduler round
};

}  // namespace
}  // namespace qld

struct qld_server {
    size_t budget = 0;
    int out_slots = 4;
    int flags = 0;
    int device = 0;
    size_t in_use = 0;
    hipStream_t compute = nullptr;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_complete;
    std::map<int, std::unique_ptr<qld::StreamRec>> streams;
    std::deque<int> pending;  // FIFO of streams waiting for budget
    int next_id = 1;
    std::deque<qld_result> results;
    std::deque<qld::Inflight> inflight;
    std::vector<hipEvent_t> free_events;
    bool stop = false;
    bool hold = false;       // qld_server_hold: launch nothing while set
    int max_inflight = 1;    // launch rounds on the device at once
    int n_inflight = 0;
    std::thread sched, complete;
    int64_t batches = 0, cycles = 0;
    int32_t max_streams = 0;
    qld_status async_error = QLD_OK;
};

namespace qld {
namespace {

int padded_w(int W, int eb) { return (int)(ceil_div(W, window_vpx(eb)) * window_vpx(eb)); }

int iq_planes(const qld_server *s, int Ms, int mode) {
    const bool keep = s->flags & QLD_SERVER_KEEP_IQ;
    return (keep ? 2 : 0) + ((keep || mode == QLD_MODE_LEARNED) && Ms > 0 ? 2 : 0);
}

int learned_ring(int Ms) { return Ms + kMaxCyclesPerJob; }

size_t stream_bytes(const qld_server *s, const qld_frame_desc *d, int M, int Ms, int mode) {
    int eb = 0;
    if (check_desc(d, &eb) != QLD_OK) return 0;
    const size_t wb = window_bytes(d, M, Ms);
    if (!wb && (size_t)d->H * d->W) return 0;
    const size_t npx = (size_t)d->H * d->W;
    const size_t stage = (size_t)kStageCycles * 4 * d->H * padded_w(d->W, eb) * eb;
    const size_t out = (size_t)s->out_slots * npx * 4;
    const size_t iq = (size_t)s->out_slots * npx * 4 * iq_planes(s, Ms, mode);
    size_t learned = 0;
    if (mode == QLD_MODE_LEARNED)
        learned = (size_t)s->out_slots * npx * 4 + npx * 8 + (size_t)learned_ring(Ms) * kCycleSumBlocks * 8 +
                  (size_t)s->out_slots * 4 + 64 + ((size_t)learned_ring(Ms) + 1) * npx * 4;
    return wb + stage + out + iq + learned;
}

void free_stream_mem(StreamRec *r) {
    if (r->win) qld_window_destroy(r->win);
    r->win = nullptr;
    if (r->stage) (void)hipFree(r->stage);
    if (r->out_amp) (void)hipFree(r->out_amp);
    if (r->out_iq) (void)hipFree(r->out_iq);
    if (r->pin) (void)hipHostFree(r->pin);
    if (r->served) (void)hipFree(r->served);
    if (r->x) (void)hipFree(r->x);
    if (r->csum) (void)hipFree(r->csum);
    if (r->pcs) (void)hipFree(r->pcs);
    if (r->gate_host) (void)hipHostFree(r->gate_host);
    r->stage = r->pin = nullptr;
    r->out_amp = nullptr;
    r->out_iq = r->Io = r->Qo = r->Iso = r->Qso = nullptr;
    r->served = r->x = r->scale = r->gate_dev = r->gate_host = nullptr;
    r->csum = r->sumS = nullptr;
    r->pcs = r->psS = nullptr;
    for (auto &e : r->pin_ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    for (auto &e : r->slot_ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    if (r->direct_ev) (void)hipEventDestroy(r->direct_ev), r->direct_ev = nullptr;
    if (r->copy) {
        (void)hipStreamSynchronize(r->copy);
        (void)hipStreamDestroy(r->copy);
        r->copy = nullptr;
    }
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
    const int planes = iq_planes(srv, r->Ms, r->mode);
    const size_t plane = (size_t)srv->out_slots * npx;
    if (e == hipSuccess && planes > 0) e = hipMalloc(&r->out_iq, plane * 4 * planes + 16);
    if (e == hipSuccess && planes > 0) {
        int32_t *q = r->out_iq;
        if (srv->flags & QLD_SERVER_KEEP_IQ) {
            r->Io = q;
            r->Qo = q + plane;
            q += 2 * plane;
        }
        if (r->Ms > 0) {
            r->Iso = q;
            r->Qso = q + plane;
        }
    }
    if (e == hipSuccess && r->mode == QLD_MODE_LEARNED) {
        r->ring = learned_ring(r->Ms);
        e = hipMalloc(&r->served, plane * 4 + 16);
        // x [H][W][2] floats, then scale, gate slots (256-byte aligned pieces).
        const size_t xb = (npx * 8 + 255) / 256 * 256, gb = ((size_t)srv->out_slots * 4 + 255) / 256 * 256;
        if (e == hipSuccess) e = hipMalloc(&r->x, xb + 256 + gb);
        if (e == hipSuccess) {
            r->scale = reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(r->x) + xb);
            r->gate_dev = reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(r->x) + xb + 256);
            e = hipMalloc(&r->csum, ((size_t)r->ring * kCycleSumBlocks + 8) * 8);
        }
        if (e == hipSuccess) {
            r->sumS = r->csum + (size_t)r->ring * kCycleSumBlocks;
            e = hipMalloc(&r->pcs, ((size_t)r->ring + 1) * npx * 4 + 16);
        }
        if (e == hipSuccess) {
            r->psS = r->pcs + (size_t)r->ring * npx;
            e = hipHostMalloc(&r->gate_host, (size_t)srv->out_slots * 4 + 16, hipHostMallocDefault);
        }
    }
    if (e == hipSuccess) e = hipHostMalloc(&r->pin, (size_t)kPinnedFrames * r->frame_bytes + 16, hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < kPinnedFrames; ++i)
        e = hipEventCreateWithFlags(&r->pin_ev[i], hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < kStageCycles; ++i)
        e = hipEventCreateWithFlags(&r->slot_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->direct_ev, hipEventDisableTiming);
    // One copy stream per camera: a small camera's frames do not queue behind
    // a large camera's (default priority, like every stream here).
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->copy, hipStreamNonBlocking);
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

// Learned work of one job, enqueued on the compute stream after the window
// update that wrote the job's short-window I/Q and plain amplitudes.
hipError_t run_learned(qld_server *srv, const LearnedJob &L) {
    StreamRec *r = L.r;
    hipStream_t s = srv->compute;
    const int64_t npx = (int64_t)r->d.H * r->d.W;
    hipError_t e = launch_cycle_sums(r->stage, r->slot_b, kStageCycles, L.stage0, L.n, r->eb, r->csum, r->ring, L.c0,
                                     kCycleSumBlocks, s);
    if (e == hipSuccess)
        e = launch_pixel_cycle_sums(r->stage, r->slot_b, r->fs_b, r->rp_b, kStageCycles, L.stage0, L.n, r->eb, r->d.H,
                                    r->d.W, r->pcs, r->ring, L.c0, s);
    for (int i = 0; i < L.n && e == hipSuccess; ++i) {
        const int64_t c = L.c0 + i;
        const int o = (L.out0 + i) % srv->out_slots;
        const float *plain = r->out_amp + (size_t)o * npx;
        float *served = r->served + (size_t)o * npx;
        const float inv_n = 1.0f / (float)std::min<int64_t>(c + 1, r->M);
        if (c + 1 >= r->Ms) {
            e = launch_window_sum(r->csum, r->ring, kCycleSumBlocks, c, r->Ms, r->sumS, s);
            if (e == hipSuccess) e = launch_pixel_window_sum(r->pcs, r->ring, npx, c, r->Ms, r->psS, s);
            if (e == hipSuccess &&
                (qld_denoise_prepare(r->Iso + (size_t)o * npx, r->Qso + (size_t)o * npx, r->psS, r->sumS, r->Ms, 1,
                                     r->d.H, r->d.W, r->x, r->scale, s) != QLD_OK ||
                 qld_denoiser_forward(L.dn, r->x, 1, nullptr, nullptr, s) != QLD_OK))
                e = hipErrorLaunchFailure;
            if (e == hipSuccess) e = launch_serve(L.y, r->scale, L.gate, plain, npx, L.thr, inv_n, served,
                                                  r->gate_dev + o, s);
        } else {
            e = launch_serve(nullptr, nullptr, nullptr, plain, npx, L.thr, inv_n, served, r->gate_dev + o, s);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->gate_host + o, r->gate_dev + o, sizeof(float), hipMemcpyDeviceToHost, s);
    }
    return e;
}

void scheduler_loop(qld_server *srv) {
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    size_t rr = 0;  // round-robin start for fairness when a launch is full
    while (true) {
        // Launch when something is ready, unless held or the device already
        // has max_inflight rounds: what lands meanwhile joins the next round.
        srv->cv_sched.wait(lk, [&] {
            if (srv->stop) return true;
            if (srv->hold || srv->n_inflight >= srv->max_inflight) return false;
            for (auto &kv : srv->streams)
                if (!kv.second->ready.empty()) return true;
            return false;
        });
        if (srv->hold || srv->n_inflight >= srv->max_inflight) {
            if (srv->stop) break;
            continue;
        }
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

        std::vector<Inflight> round;
        for (auto &g : groups) {
            WinBatch b{};
            std::vector<CycleRef> refs;
            std::vector<LearnedJob> ljobs;
            std::vector<hipEvent_t> waits;
            int tiles = 0;
            for (StreamRec *r : g.second) {
                if (b.n_jobs == kMaxJobs) break;
                WinJob &J = b.job[b.n_jobs];
                const int64_t k0 = r->ready.front();
                const int slot0 = (int)(k0 % kStageCycles);
                const bool fresh = r->slot_reset[slot0];
                // A job's cycles each need their own output slot.
                const int max_n = std::min(kMaxCyclesPerJob, srv->out_slots);
                int n = 0;
                while (n < (int)r->ready.size() && n < max_n) {
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
                J.Io = r->Io;
                J.Qo = r->Qo;
                J.Iso = r->Iso;
                J.Qso = r->Qso;
                (void)npx;
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
                                            (int)(k % srv->out_slots), r->gate_thr});
                }
                if (r->mode == QLD_MODE_LEARNED)
                    ljobs.push_back(LearnedJob{r, r->dn, r->dn_y, r->dn_gate, r->gate_thr, c0, n, J.out0, slot0});
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
            for (const LearnedJob &L : ljobs)
                if (e == hipSuccess) e = run_learned(srv, L);
            if (e == hipSuccess && ev) e = hipEventRecord(ev, srv->compute);
            lk.lock();
            if (e != hipSuccess || !ev) {
                srv->async_error = QLD_E_DEVICE;
                set_error("server launch failed: %s", hipGetErrorString(e));
            }
            srv->batches++;
            srv->max_streams = std::max<int32_t>(srv->max_streams, b.n_jobs);
            round.push_back(Inflight{ev, std::move(refs), false});
        }
        if (!round.empty()) {
            round.back().round_end = true;
            for (Inflight &f : round) srv->inflight.push_back(std::move(f));
            srv->n_inflight++;
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
            res.amp_plain = res.amp;
            res.H = r->d.H;
            res.W = r->d.W;
            if (r->mode == QLD_MODE_LEARNED) {
                res.amp = r->served + (size_t)c.out_slot * r->d.H * r->d.W;
                res.gate = r->gate_host[c.out_slot];
                res.learned = (res.gate == res.gate && res.gate <= c.gate_thr) ? 1 : 0;
            }
            res.seq = c.k;
            srv->results.push_back(res);
            r->done++;
            srv->cycles++;
        }
        if (f.round_end) {
            srv->n_inflight--;
            srv->cv_sched.notify_one();
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
    const qld_status st = check_hip(hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking), "compute stream");
    if (st != QLD_OK) {
        delete s;
        return st;
    }
    s->sched = std::thread(scheduler_loop, s);
    s->complete = std::thread(completion_loop, s);
    *out = s;
    return QLD_OK;
}

extern "C" size_t qld_server_stream_bytes(const qld_server *s, const qld_frame_desc *d, int32_t M_cycles,
                                          int32_t M_short, int32_t mode) {
    if (!s || (mode != QLD_MODE_PLAIN && mode != QLD_MODE_LEARNED)) return 0;
    return stream_bytes(s, d, M_cycles, M_short, mode);
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
    if (M_cycles < 1 || M_short < 0 || M_short > M_cycles || (mode != QLD_MODE_PLAIN && mode != QLD_MODE_LEARNED) ||
        (mode == QLD_MODE_LEARNED && M_short < 1)) {
        set_error("invalid window M=%d short=%d mode=%d", M_cycles, M_short, mode);
        return QLD_E_INVAL;
    }
    if ((uint64_t)M_cycles * ((1ull << d->bits) - 1) >= (1ull << 31)) {
        set_error("M=%d cycles of %d-bit data could overflow int32", M_cycles, d->bits);
        return QLD_E_OVERFLOW;
    }
    const size_t need = stream_bytes(s, d, M_cycles, M_short, mode);
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

extern "C" qld_status qld_stream_set_denoiser(qld_server *s, int32_t stream_id, qld_denoiser *dn,
                                             float gate_threshold) {
    clear_error();
    if (!s || !dn || gate_threshold != gate_threshold) {
        set_error("server and denoiser must be non-NULL and the threshold a number");
        return QLD_E_INVAL;
    }
    int32_t H = 0, W = 0, mb = 0;
    QLD_TRY(qld_denoiser_info(dn, &H, &W, &mb));
    void *y = nullptr, *g = nullptr;
    int64_t cnt = 0;
    QLD_TRY(qld_denoiser_tensor(dn, 4, &y, &cnt));
    QLD_TRY(qld_denoiser_tensor(dn, 8, &g, &cnt));
    std::lock_guard<std::mutex> lk(s->mu);
    StreamRec *r = find_stream(s, stream_id);
    if (!r || r->state == QLD_STREAM_CLOSED || r->mode != QLD_MODE_LEARNED) {
        set_error("stream %d is not an open LEARNED stream", stream_id);
        return r ? QLD_E_STATE : QLD_E_INVAL;
    }
    if (H != r->d.H || W != r->d.W) {
        set_error("denoiser is %dx%d, stream is %dx%d", H, W, r->d.H, r->d.W);
        return QLD_E_SHAPE;
    }
    r->dn = dn;
    r->dn_y = static_cast<const float *>(y);
    r->dn_gate = static_cast<const float *>(g);
    r->gate_thr = gate_threshold;
    return QLD_OK;
}

namespace qld {
namespace {

// The stream a submit goes to, if it may take frames now (mu held).
qld_status open_for_submit(qld_server *s, int32_t stream_id, StreamRec **out) {
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
    if (r->mode == QLD_MODE_LEARNED && !r->dn) {
        set_error("stream %d is LEARNED and has no denoiser", stream_id);
        return QLD_E_STATE;
    }
    *out = r;
    return QLD_OK;
}

// Back-pressure before the first frame of the stream's next cycle: its
// device staging slot must have been consumed (mu held; waits).  While the
// server is held nothing is launched, so instead of waiting for ever this
// returns QLD_E_AGAIN and the submit takes nothing.
qld_status wait_slot(qld_server *s, StreamRec *r, std::unique_lock<std::mutex> &lk) {
    const int64_t k = r->submitted;
    auto slot_free = [&] { return r->done > k - kStageCycles; };
    s->cv_done.wait(lk, [&] { return slot_free() || s->async_error != QLD_OK || s->hold; });
    if (s->async_error != QLD_OK) return s->async_error;
    if (!slot_free()) {
        set_error("stream %d: every staging slot holds a cycle the held server has not launched", r->id);
        return QLD_E_AGAIN;
    }
    return QLD_OK;
}

// True if p lies in page-locked host memory (hipHostMalloc), which the copy
// engine reads directly.  Pageable memory makes the query fail; the error is
// cleared so that the next call does not report it.
bool page_locked(const void *p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) == hipSuccess) return at.type == hipMemoryTypeHost;
    (void)hipGetLastError();
    return false;
}

// Copies n frames (phases phase .. phase + n - 1 of the stream's next cycle)
// to the stream's device staging with one host-to-device copy on the
// stream's own copy stream; the cycle goes to the scheduler once its last frame is in.  Frames
// in pageable memory are first copied into the stream's pinned staging (so
// the caller may reuse its buffer at once); frames already in page-locked
// memory are copied straight from the caller's buffer, and the call waits for
// that copy before it returns (same ownership rule, one copy fewer).  mu is
// held on entry and exit and released around the copies.
qld_status stage_frames(qld_server *s, StreamRec *r, std::unique_lock<std::mutex> &lk, const void *host, int phase,
                        int n, int64_t cam_cycle, uint64_t t_arrival_ns) {
    const int64_t k = r->submitted;
    const int slot = (int)(k % kStageCycles);
    const bool direct = page_locked(host);
    const int p0 = (int)(k % kPinnedCycles) * 4 + phase;
    bool used[4] = {};
    hipEvent_t pev[4] = {};
    if (!direct) {
        for (int i = 0; i < n; ++i) {
            used[i] = r->pin_used[p0 + i];
            r->pin_used[p0 + i] = true;
            pev[i] = r->pin_ev[p0 + i];
        }
    }
    uint8_t *pin = r->pin + (size_t)p0 * r->frame_bytes;
    uint8_t *dst = r->stage + (size_t)slot * r->slot_b + (size_t)phase * r->fs_b;
    const size_t row = (size_t)r->d.W * r->eb;
    lk.unlock();

    hipError_t e = hipSuccess;
    if (direct) {
        e = hipMemcpy2DAsync(dst, (size_t)r->rp_b, host, row, row, (size_t)n * r->d.H, hipMemcpyHostToDevice,
                             r->copy);
        if (e == hipSuccess && phase + n == 4) e = hipEventRecord(r->slot_ev[slot], r->copy);
        if (e == hipSuccess) e = hipEventRecord(r->direct_ev, r->copy);
        // The caller's buffer is free again once the copy is done.  Waiting
        // before the cycle is queued also keeps a cycle whose copy is still in
        // flight out of the next batched launch, which would hold every other
        // stream's image in that launch until this copy lands.
        if (e == hipSuccess) e = hipEventSynchronize(r->direct_ev);
    } else {
        for (int i = 0; i < n && e == hipSuccess; ++i)
            if (used[i]) e = hipEventSynchronize(pev[i]);   // the pinned frame's previous copy is done
        if (e == hipSuccess) {
            memcpy(pin, host, (size_t)n * r->frame_bytes);
            // The staged frames of a cycle are consecutive [H][Wp] planes, so n
            // frames are one copy of n * H rows.
            e = hipMemcpy2DAsync(dst, (size_t)r->rp_b, pin, row, row, (size_t)n * r->d.H, hipMemcpyHostToDevice,
                                 r->copy);
        }
        for (int i = 0; i < n && e == hipSuccess; ++i) e = hipEventRecord(pev[i], r->copy);
        if (e == hipSuccess && phase + n == 4) e = hipEventRecord(r->slot_ev[slot], r->copy);
    }

    lk.lock();
    if (e != hipSuccess) {
        set_error("frame copy failed: %s", hipGetErrorString(e));
        return QLD_E_DEVICE;
    }
    r->cur = phase + n;
    if (r->cur == 4) {
        r->slot_tarr[slot] = t_arrival_ns;
        r->slot_cam_cycle[slot] = cam_cycle;
        r->slot_reset[slot] = r->reset_next;
        r->reset_next = false;
        r->ready.push_back(k);
        r->submitted++;
        r->cur = 0;
        s->cv_sched.notify_one();
    }
    return QLD_OK;
}

}  // namespace
}  // namespace qld

extern "C" qld_status qld_stream_submit(qld_server *s, int32_t stream_id, const void *host_frame,
                                        int64_t frame_index, uint64_t t_arrival_ns) {
    clear_error();
    if (!s || !host_frame) {
        set_error("server and host_frame must be non-NULL");
        return QLD_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    StreamRec *r = nullptr;
    QLD_TRY(open_for_submit(s, stream_id, &r));
    if (frame_index < r->next_frame) {
        set_error("frame index %lld < expected %lld", (long long)frame_index, (long long)r->next_frame);
        return QLD_E_INVAL;
    }
    // What the frame does is decided before any state changes, so that a
    // submit returning QLD_E_AGAIN has taken nothing and can be repeated.
    // A gap loses the phase alignment: the partial cycle is dropped, frames
    // are skipped until a cycle starts, and the window restarts.
    const bool gap = frame_index > r->next_frame;
    const int phase = (int)(frame_index & 3);
    bool dropping = gap || r->dropping;
    int cur = gap ? 0 : r->cur;
    bool take = true;
    if (dropping) {
        if (phase != 0) take = false;   // wait for the first frame of a cycle
        else dropping = false;
    }
    if (take && phase != cur) {
        // Stream started mid-cycle (first frame index not a multiple of 4).
        cur = 0;
        if (phase != 0) take = false;
    }
    if (take && phase == 0) QLD_TRY(wait_slot(s, r, lk));
    qld_status ret = QLD_OK;
    if (gap) {
        r->reset_next = true;
        ret = QLD_E_GAP;
        set_error("frame index jumped from %lld to %lld: window reset", (long long)r->next_frame,
                  (long long)frame_index);
    }
    r->next_frame = frame_index + 1;
    r->dropping = dropping;
    r->cur = cur;
    if (!take) return ret;
    const qld_status st = stage_frames(s, r, lk, host_frame, phase, 1, frame_index >> 2, t_arrival_ns);
    return st != QLD_OK ? st : ret;
}

extern "C" qld_status qld_stream_submit_cycle(qld_server *s, int32_t stream_id, const void *host_frames,
                                              int64_t first_frame_index, uint64_t t_arrival_ns) {
    clear_error();
    if (!s || !host_frames) {
        set_error("server and host_frames must be non-NULL");
        return QLD_E_INVAL;
    }
    if (first_frame_index < 0 || first_frame_index % 4 != 0) {
        set_error("first_frame_index %lld is not a multiple of 4", (long long)first_frame_index);
        return QLD_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    StreamRec *r = nullptr;
    QLD_TRY(open_for_submit(s, stream_id, &r));
    if (first_frame_index < r->next_frame) {
        set_error("frame index %lld < expected %lld", (long long)first_frame_index, (long long)r->next_frame);
        return QLD_E_INVAL;
    }
    const bool gap = first_frame_index > r->next_frame;
    QLD_TRY(wait_slot(s, r, lk));
    qld_status ret = QLD_OK;
    if (gap) {
        r->reset_next = true;
        ret = QLD_E_GAP;
        set_error("frame index jumped from %lld to %lld: window reset", (long long)r->next_frame,
                  (long long)first_frame_index);
    }
    r->next_frame = first_frame_index + 4;
    r->dropping = false;
    r->cur = 0;
    const qld_status st = stage_frames(s, r, lk, host_frames, 0, 4, first_frame_index >> 2, t_arrival_ns);
    return st != QLD_OK ? st : ret;
}

extern "C" qld_status qld_server_hold(qld_server *s, int32_t on) {
    clear_error();
    if (!s) return QLD_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->hold = on != 0;
    }
    s->cv_sched.notify_all();
    s->cv_done.notify_all();   // a submit waiting for a staging slot re-checks
    return QLD_OK;
}

extern "C" qld_status qld_server_set_max_inflight(qld_server *s, int32_t n) {
    clear_error();
    if (!s || n < 1 || n > kMaxInflight) {
        set_error("max_inflight must be in 1..%d", kMaxInflight);
        return QLD_E_INVAL;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->max_inflight = n;
    }
    s->cv_sched.notify_all();
    return QLD_OK;
}

extern "C" qld_status qld_stream_result_valid(qld_server *s, const qld_result *res, int32_t *valid) {
    clear_error();
    if (!s || !res || !valid) return QLD_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    StreamRec *r = find_stream(s, res->stream_id);
    // The result's output slot is rewritten by the stream's cycle
    // seq + out_slots; cycles are launched in order.
    *valid = (r && r->state != QLD_STREAM_CLOSED && res->seq >= 0 && res->seq < r->launched &&
              r->launched <= res->seq + s->out_slots)
                 ? 1
                 : 0;
    return QLD_OK;
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
    s->hold = false;
    s->cv_sched.notify_all();
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
    s->hold = false;
    s->cv_sched.notify_all();
    s->cv_done.wait(lk, [&] { return r->done >= r->submitted || s->async_error != QLD_OK; });
    // Results already published keep pointing at this stream's output slots:
    // drop them so nobody reads freed memory.
    s->results.erase(std::remove_if(s->results.begin(), s->results.end(),
                                     [&](const qld_result &q) { return q.stream_id == stream_id; }),
                     s->results.end());
    lk.unlock();
    if (r->copy) (void)hipStreamSynchronize(r->copy);
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
        s->hold = false;
        s->cv_sched.notify_all();
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
    for (auto &kv : s->streams) free_stream_mem(kv.second.get());   // each stream's copies finish first
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    for (auto &f : s->inflight)
        if (f.ev) (void)hipEventDestroy(f.ev);
    (void)hipStreamDestroy(s->compute);
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
    const size_t slot = (size_t)(res->amp_plain - r->out_amp) / npx;
    if (slot >= (size_t)s->out_slots) {
        set_error("result does not belong to stream %d", res->stream_id);
        return QLD_E_INVAL;
    }
    if (I) *I = r->Io ? r->Io + slot * npx : nullptr;
    if (Q) *Q = r->Qo ? r->Qo + slot * npx : nullptr;
    if (Is) *Is = r->Iso ? r->Iso + slot * npx : nullptr;
    if (Qs) *Qs = r->Qso ? r->Qso + slot * npx : nullptr;
    return QLD_OK;
}
