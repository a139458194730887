// Serving sessions: continuing per-channel streams with HBM-resident state and
// continuous batching.
//
// Every channel owns a device-resident state record (AEQ taps, CDC and AEQ
// overlap tails).  Requests are segments of a channel's stream (multiples of
// 32 instants = one CDC hop = one AEQ block).  A scheduler thread issues
// "ticks": each tick advances every active request by at most chunk_blocks
// blocks with one batched CDC launch and one batched AEQ launch, so requests
// that arrive while others run join at the next tick and long requests never
// hold short ones back.  A request of a channel may follow the previous one of
// the same channel in the very next tick: the launches are ordered on one
// stream and the state record carries the history.  A completion thread
// retires ticks in order and stamps request latencies.  Host-buffer requests
// are staged through a first-fit pool inside the session's HBM budget; a
// request that does not fit waits (admission by footprint).  Their PCIe copies
// run on two copy streams of their own, so a tick's input upload and the
// previous tick's result download overlap the kernels in between.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fnt_common.hpp"
#include "fnt_internal.hpp"

using namespace fnti;

namespace {

struct DevState {               // one per channel, FNT_STATE_BYTES in device memory
    int16_t taps[256];
    int8_t cdc_tail[128];
    int8_t aeq_tail[64];
    uint64_t position;          // instants consumed (host keeps the copy that counts)
    uint8_t pad[768 - 512 - 128 - 64 - 8];
};
static_assert(sizeof(DevState) == FNT_STATE_BYTES, "state record size");

enum ReqStatus { QUEUED, ACTIVE, DONE, CANCELLED };

struct Request {
    uint64_t ticket = 0;
    uint32_t ch = 0;
    uint32_t flags = 0;
    const int8_t *in = nullptr;     // device input (caller's or staged)
    int16_t *out = nullptr;         // device output (caller's or staged)
    const int8_t *host_in = nullptr;
    int16_t *host_out = nullptr;
    uint64_t n = 0;                 // instants
    uint64_t blocks = 0;            // n / 32
    uint64_t issued = 0;            // blocks already placed in ticks
    uint64_t arrival_ns = 0;
    uint64_t pool_off = 0, pool_len = 0;
    bool staged = false;
    ReqStatus status = QUEUED;
};

struct Channel {
    bool registered = false;
    bool in_rr = false;             // listed in the scheduler's round robin
    fnt_cdc_params cdc{};
    fnt_aeq_params aeq{};
    std::deque<uint64_t> queue;     // tickets in submission order (queued or active)
    uint64_t position = 0;
    // The AEQ history has two device copies: a tick reads one and writes the
    // other, so no workgroup of a tick can read a history that another
    // workgroup of the same tick has already replaced (the two polarisation
    // halves of a channel may run as separate workgroups).  tail_sel names the
    // copy holding the current history: 0 = DevState::aeq_tail, 1 = the
    // session's aeq_tail_alt record of the channel.
    int tail_sel = 0;
    uint64_t last_seq = 0;          // last tick that advanced the channel
};

// First-fit allocator over [0, size) with coalescing.
class Pool {
   public:
    void init(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
    }
    bool alloc(uint64_t len, uint64_t *off) {
        len = (len + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *off = it->first;
                uint64_t rest = it->second - len, start = it->first + len;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t len) {
        len = (len + 255) & ~255ull;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }

   private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0;
};

struct TickSlot {
    CdcItem *cdc_host = nullptr;    // pinned
    AeqItem *aeq_host = nullptr;    // pinned
    CdcItem *cdc_dev = nullptr;
    AeqItem *aeq_dev = nullptr;
    int8_t *scratch = nullptr;      // decimated symbols, max_active * chunk * 64 bytes
    hipEvent_t done = nullptr;      // kernels and result downloads of the tick finished
    hipEvent_t staged = nullptr;    // input uploads of requests admitted in the tick finished
    hipEvent_t computed = nullptr;  // kernels of the tick finished
    bool busy = false;
    std::vector<uint64_t> finishing;   // tickets whose last block is in this tick
    uint64_t seq = 0;
};

constexpr int kSlots = 3;

}  // namespace

struct fnt_session {
    fnt_session_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;      // tick kernels, in order
    hipStream_t copy_in = nullptr;     // host-to-device staging of admitted requests
    hipStream_t copy_out = nullptr;    // device-to-host results of finished requests
    DevState *dstate = nullptr;
    int8_t *aeq_tail_alt = nullptr;    // [max_channels][64]: second copy of each AEQ history
    int8_t *pool_base = nullptr;
    Pool pool;
    int *err = nullptr;
    std::vector<Channel> chans;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<uint32_t> rr;          // channels with queued work, round-robin order
    TickSlot slots[kSlots];
    uint64_t next_ticket = 1;
    uint64_t tick_seq = 0;
    uint64_t retired_seq = 0;          // ticks retire in launch order: every seq <= this has ended
    std::deque<int> inflight;          // slot indices in launch order

    std::mutex mu;
    std::condition_variable cv_work;   // scheduler: new work or a free slot
    std::condition_variable cv_done;   // waiters: a request completed
    std::condition_variable cv_inflight;  // completion thread: a tick was launched
    bool stop = false;
    int fatal = 0;
    std::string fatal_msg;
    std::thread sched, compl_;

    // statistics
    fnt_session_stats st{};
    std::vector<double> lat_us;
    uint64_t first_arrival = UINT64_MAX, last_completion = 0;
};

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void set_fatal(fnt_session *s, const char *what, hipError_t e) {
    if (!s->fatal) {
        s->fatal = FNT_E_DEVICE;
        s->fatal_msg = std::string(what) + ": " + hipGetErrorString(e);
    }
}

// Bytes of pool staging for a host-buffer request of n instants: the input
// (n * 4) rounded to 256, then the output (n / 2 symbols * 8 bytes).
uint64_t staging_bytes(uint64_t n) { return ((n * 4 + 255) & ~255ull) + n * 4; }

// Build one tick's work (called with the lock held).  Channels served in this
// tick move behind the ones that were not, so every channel makes progress.
// Input uploads of newly admitted host-buffer requests are queued on the
// upload stream; *uploads tells whether there were any.
int build_tick(fnt_session *s, TickSlot &slot, bool *uploads) {
    *uploads = false;
    const uint32_t chunk = s->cfg.chunk_blocks;
    const uint32_t cap = s->cfg.max_active;
    int nitems = 0;
    uint64_t block0 = 0, chunk0 = 0;
    slot.finishing.clear();
    std::vector<uint32_t> served, waiting;
    served.reserve(s->rr.size());
    waiting.reserve(s->rr.size());
    for (uint32_t c : s->rr) {
        Channel &ch = s->chans[c];
        if ((uint32_t)nitems == cap) {
            waiting.push_back(c);
            continue;
        }
        while (!ch.queue.empty() && s->reqs[ch.queue.front()].status == CANCELLED)
            ch.queue.pop_front();
        if (ch.queue.empty()) {
            ch.in_rr = false;
            continue;
        }
        Request &r = s->reqs[ch.queue.front()];
        if (r.status == QUEUED) {
            if (r.flags & FNT_SUBMIT_HOST) {
                uint64_t len = staging_bytes(r.n), off;
                if (!s->pool.alloc(len, &off)) {  // does not fit now: wait for memory
                    waiting.push_back(c);
                    continue;
                }
                r.pool_off = off;
                r.pool_len = len;
                r.in = s->pool_base + off;
                r.out = reinterpret_cast<int16_t *>(s->pool_base + off + ((r.n * 4 + 255) & ~255ull));
                hipError_t e = hipMemcpyAsync((void *)r.in, r.host_in, r.n * 4, hipMemcpyHostToDevice,
                                              s->copy_in);
                if (e != hipSuccess) set_fatal(s, "session: stage input", e);
                r.staged = true;
                *uploads = true;
            }
            r.status = ACTIVE;
        }
        uint64_t nb = std::min<uint64_t>(chunk, r.blocks - r.issued);
        DevState *st = s->dstate + c;
        CdcItem &ci = slot.cdc_host[nitems];
        fill_cdc_item(ci, r.in + r.issued * 32 * 4, nb * 32, &ch.cdc);
        ci.hist = st->cdc_tail;
        ci.a_out = slot.scratch + (uint64_t)nitems * chunk * 16 * 4;
        ci.block0 = block0;
        ci.chunk0 = chunk0;
        block0 += nb;
        chunk0 += cdc_chunks(ci.n);
        AeqItem &ai = slot.aeq_host[nitems];
        fill_aeq_item(ai, ci.a_out, nb * 16, st->taps, &ch.aeq, r.out + r.issued * 16 * 4);
        ai.block0 = ch.position / 32;   // the stream's AEQ blocks so far (32 instants each)
        int8_t *tails[2] = {st->aeq_tail, s->aeq_tail_alt + (uint64_t)c * 64};
        ai.hist_in = tails[ch.tail_sel];
        ai.hist_out = tails[ch.tail_sel ^ 1];
        ch.tail_sel ^= 1;
        ch.last_seq = s->tick_seq + 1;   // the seq this tick receives when it is issued
        ai.cdc_in = ci.in;
        ai.cdc_n = ci.n;
        ai.cdc_tail = st->cdc_tail;
        r.issued += nb;
        ch.position += nb * 32;
        ++nitems;
        if (r.issued == r.blocks) {   // fully issued: the next request may follow next tick
            slot.finishing.push_back(r.ticket);
            ch.queue.pop_front();
        }
        if (ch.queue.empty()) ch.in_rr = false;
        else served.push_back(c);
    }
    waiting.insert(waiting.end(), served.begin(), served.end());
    s->rr.swap(waiting);
    return nitems;
}

// AEQ form for a tick of `nitems` chains of equal length: the one with the
// shortest tick, per block max(serial latency, work / issue rate), from the
// forms' measured per-block latency (us, one chain alone) and VALU instructions
// per chain-block on MI355X (1024 SIMDs, 0.6e12 wave instructions/s, taken at
// 70 % efficiency).
int tick_form(int nitems) {
    struct Form { int code; double lat_us, instr; };
    static const Form forms[] = {{4, 0.70, 1472}, {2, 0.84, 1020}, {1, 1.08, 774}, {3, 2.05, 740}, {0, 2.70, 600}};
    int best = 4;
    double best_t = 1e30;
    for (const Form &f : forms) {
        const double t = std::max(f.lat_us, nitems * f.instr / (0.7 * 0.6e12) * 1e6);
        if (t < best_t) {
            best_t = t;
            best = f.code;
        }
    }
    return best;
}

void scheduler_main(fnt_session *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        int slot_idx = -1;
        for (int k = 0; k < kSlots; ++k)
            if (!s->slots[k].busy) {
                slot_idx = k;
                break;
            }
        // keep at most two ticks queued ahead so late arrivals join soon
        if (slot_idx < 0 || s->inflight.size() >= 2 || s->rr.empty() || s->fatal) {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        TickSlot &slot = s->slots[slot_idx];
        bool uploads = false;
        int nitems = build_tick(s, slot, &uploads);
        if (nitems == 0) {
            s->cv_work.wait_for(lk, std::chrono::microseconds(200));
            continue;
        }
        slot.busy = true;
        slot.seq = ++s->tick_seq;
        // host-buffer requests that finish in this tick copy their output back
        std::vector<std::pair<int16_t *, std::pair<const int16_t *, uint64_t>>> d2h;
        for (uint64_t t : slot.finishing) {
            Request &r = s->reqs[t];
            if (r.staged) d2h.push_back({r.host_out, {r.out, (r.n / 2) * 8}});
        }
        lk.unlock();
        hipStream_t st = s->stream;
        hipError_t e = hipSuccess;
        if (uploads) {   // the tick's kernels read the inputs just queued for upload
            e = hipEventRecord(slot.staged, s->copy_in);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, slot.staged, 0);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(slot.cdc_dev, slot.cdc_host, nitems * sizeof(CdcItem),
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot.aeq_dev, slot.aeq_host, nitems * sizeof(AeqItem),
                               hipMemcpyHostToDevice, st);
        uint64_t total_blocks = 0, total_chunks = 0;
        for (int k = 0; k < nitems; ++k) {
            total_blocks += cdc_blocks(slot.cdc_host[k].n);
            total_chunks += cdc_chunks(slot.cdc_host[k].n);
        }
        if (e == hipSuccess) {
            int wpg, bpw;
            default_cdc_schedule(total_blocks, &wpg, &bpw);
            e = run_cdc(slot.cdc_dev, nitems, CdcItem{}, total_blocks, total_chunks, wpg, bpw, false, s->err, st);
        }
        if (e == hipSuccess) {
            const int form = s->cfg.aeq_form >= 0 ? s->cfg.aeq_form : tick_form(nitems);
            e = launch_aeq(slot.aeq_dev, nitems, AeqItem{}, 0, form, s->err, st);
        }
        if (d2h.empty()) {
            if (e == hipSuccess) e = hipEventRecord(slot.done, st);
        } else {         // downloads wait for this tick's kernels only, not for later ticks
            if (e == hipSuccess) e = hipEventRecord(slot.computed, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(s->copy_out, slot.computed, 0);
            for (auto &c : d2h)
                if (e == hipSuccess)
                    e = hipMemcpyAsync(c.first, c.second.first, c.second.second, hipMemcpyDeviceToHost,
                                       s->copy_out);
            if (e == hipSuccess) e = hipEventRecord(slot.done, s->copy_out);
        }
        lk.lock();
        if (e != hipSuccess) set_fatal(s, "session: tick launch", e);
        s->st.ticks++;
        s->inflight.push_back(slot_idx);
        s->cv_inflight.notify_all();
    }
}

void completion_main(fnt_session *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (s->inflight.empty() && !s->stop) s->cv_inflight.wait(lk);
        if (s->inflight.empty() && s->stop) break;
        int k = s->inflight.front();
        TickSlot &slot = s->slots[k];
        lk.unlock();
        hipError_t e = hipEventSynchronize(slot.done);
        uint64_t t = now_ns();
        lk.lock();
        if (e != hipSuccess) set_fatal(s, "session: tick completion", e);
        s->inflight.pop_front();
        s->retired_seq = slot.seq;
        for (uint64_t tk : slot.finishing) {
            auto it = s->reqs.find(tk);
            if (it == s->reqs.end()) continue;
            Request &r = it->second;
            r.status = DONE;
            if (r.pool_len) s->pool.release(r.pool_off, r.pool_len);
            r.pool_len = 0;
            double us = (double)(t - std::min(t, r.arrival_ns)) / 1e3;
            s->lat_us.push_back(us);
            s->st.completed++;
            s->st.instants_done += r.n;
            s->first_arrival = std::min(s->first_arrival, r.arrival_ns);
            s->last_completion = std::max(s->last_completion, t);
        }
        slot.busy = false;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

int check_fatal(fnt_session *s) {
    if (s->fatal) return fail(s->fatal, "%s", s->fatal_msg.c_str());
    return FNT_OK;
}

// Wait (lock held through lk) until the last tick that advanced channel ch has
// retired, so its kernels no longer read or write the channel's state.  A
// request leaves its channel's queue when its last block is placed in a tick,
// before that tick runs, so an empty queue alone does not make the state free.
int wait_channel_ticks(fnt_session *s, std::unique_lock<std::mutex> &lk, uint32_t ch) {
    while (s->retired_seq < s->chans[ch].last_seq) {
        if (s->fatal) return check_fatal(s);
        s->cv_done.wait_for(lk, std::chrono::milliseconds(5));
    }
    return FNT_OK;
}

bool channel_idle(fnt_session *s, uint32_t ch) {
    for (uint64_t t : s->chans[ch].queue) {
        auto it = s->reqs.find(t);
        if (it != s->reqs.end() && (it->second.status == QUEUED || it->second.status == ACTIVE)) return false;
    }
    return true;
}

void free_session(fnt_session *s) {
    for (auto &sl : s->slots) {
        if (sl.cdc_host) (void)hipHostFree(sl.cdc_host);
        if (sl.aeq_host) (void)hipHostFree(sl.aeq_host);
        if (sl.cdc_dev) (void)hipFree(sl.cdc_dev);
        if (sl.aeq_dev) (void)hipFree(sl.aeq_dev);
        if (sl.scratch) (void)hipFree(sl.scratch);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.staged) (void)hipEventDestroy(sl.staged);
        if (sl.computed) (void)hipEventDestroy(sl.computed);
    }
    if (s->dstate) (void)hipFree(s->dstate);
    if (s->aeq_tail_alt) (void)hipFree(s->aeq_tail_alt);
    if (s->pool_base) (void)hipFree(s->pool_base);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy_in) (void)hipStreamDestroy(s->copy_in);
    if (s->copy_out) (void)hipStreamDestroy(s->copy_out);
    delete s;
}

}  // namespace

extern "C" {

uint64_t fnt_now_ns(void) { return now_ns(); }

int fnt_session_create(fnt_session **out, const fnt_session_config *cfg) {
    if (!out || !cfg) return fail(FNT_E_INVAL, "session: NULL argument");
    *out = nullptr;
    if (cfg->max_channels == 0 || cfg->max_channels > (1u << 20))
        return fail(FNT_E_INVAL, "session: max_channels %u outside [1, 2^20]", cfg->max_channels);
    fnt_session *s = new fnt_session();
    s->cfg = *cfg;
    if (s->cfg.chunk_blocks == 0) s->cfg.chunk_blocks = 512;
    if (s->cfg.chunk_blocks > 4096) {
        delete s;
        return fail(FNT_E_INVAL, "session: chunk_blocks %u > 4096", cfg->chunk_blocks);
    }
    if (cfg->aeq_form < -1 || cfg->aeq_form > 5) {
        delete s;
        return fail(FNT_E_INVAL, "session: aeq_form %d outside [-1, 5]", cfg->aeq_form);
    }
    if (s->cfg.max_active == 0 || s->cfg.max_active > s->cfg.max_channels)
        s->cfg.max_active = s->cfg.max_channels;
    s->device = cfg->device;
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "session: hipSetDevice");
    }
    int rc = device_err_flag(&s->err);
    if (rc) {
        delete s;
        return rc;
    }
    const uint64_t scratch_bytes = (uint64_t)s->cfg.max_active * s->cfg.chunk_blocks * 64;
    const uint64_t fixed = (uint64_t)kSlots * scratch_bytes + (uint64_t)s->cfg.max_channels * (sizeof(DevState) + 64);
    if (cfg->hbm_budget_bytes < fixed) {
        delete s;
        return fail(FNT_E_NOMEM, "session: budget %llu below the fixed %llu bytes",
                    (unsigned long long)cfg->hbm_budget_bytes, (unsigned long long)fixed);
    }
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_in, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_out, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s->dstate, (size_t)s->cfg.max_channels * sizeof(DevState));
    if (e == hipSuccess) e = hipMalloc(&s->aeq_tail_alt, (size_t)s->cfg.max_channels * 64);
    const uint64_t pool = cfg->hbm_budget_bytes - fixed;
    if (e == hipSuccess && pool) e = hipMalloc(&s->pool_base, pool);
    for (int k = 0; k < kSlots && e == hipSuccess; ++k) {
        TickSlot &sl = s->slots[k];
        size_t ni = s->cfg.max_active;
        e = hipHostMalloc((void **)&sl.cdc_host, ni * sizeof(CdcItem), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.aeq_host, ni * sizeof(AeqItem), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&sl.cdc_dev, ni * sizeof(CdcItem));
        if (e == hipSuccess) e = hipMalloc(&sl.aeq_dev, ni * sizeof(AeqItem));
        if (e == hipSuccess) e = hipMalloc(&sl.scratch, scratch_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.staged, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.computed, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        free_session(s);
        (void)hipGetLastError();       // the failed call must not surface in the caller's next launch check
        return fail(FNT_E_NOMEM, "session: allocation: %s", hipGetErrorString(e));
    }
    s->pool.init(pool);
    s->chans.resize(s->cfg.max_channels);
    s->st = fnt_session_stats{};
    s->sched = std::thread(scheduler_main, s);
    s->compl_ = std::thread(completion_main, s);
    *out = s;
    return FNT_OK;
}

int fnt_session_add_channel(fnt_session *s, uint32_t ch, const fnt_cdc_params *cp,
                            const fnt_aeq_params *ap, const int16_t *host_init_taps) {
    if (!s) return fail(FNT_E_INVAL, "session: NULL");
    int rc = validate_cdc(cp);
    if (rc) return rc;
    if ((rc = validate_aeq(ap))) return rc;
    if (cp->decim_phase != 0) return fail(FNT_E_INVAL, "session: decim_phase must be 0");
    if (ch >= s->cfg.max_channels) return fail(FNT_E_STATE, "session: channel %u out of range", ch);
    DevState h;
    std::memset(&h, 0, sizeof h);
    if (host_init_taps) {
        for (int i = 0; i < 256; ++i) {
            if (host_init_taps[i] < -8192 || host_init_taps[i] > 8191)
                return fail(FNT_E_RANGE, "session: initial tap %d = %d outside 14 bit", i, host_init_taps[i]);
            h.taps[i] = host_init_taps[i];
        }
    } else {
        for (int d = 0; d < 4; ++d) h.taps[(d * 4 + d) * 16 + 8] = 4096;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (!channel_idle(s, ch)) return fail(FNT_E_STATE, "session: channel %u busy", ch);
    if ((rc = wait_channel_ticks(s, lk, ch))) return rc;
    Channel &c = s->chans[ch];
    c.registered = true;
    c.cdc = *cp;
    c.aeq = *ap;
    c.position = 0;
    c.tail_sel = 0;
    lk.unlock();
    hipError_t e = hipMemcpy(s->dstate + ch, &h, sizeof h, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "session: upload channel state");
    return FNT_OK;
}

static int submit_locked(fnt_session *s, uint32_t ch, const int8_t *in, uint64_t n, int16_t *out,
                         uint32_t flags, uint64_t arrival_ns, uint64_t *ticket) {
    if (ch >= s->cfg.max_channels || !s->chans[ch].registered)
        return fail(FNT_E_STATE, "session: channel %u not registered", ch);
    if (n == 0 || n % 32) return fail(FNT_E_INVAL, "session: n = %llu is not a positive multiple of 32",
                                      (unsigned long long)n);
    if (!in || !out) return fail(FNT_E_INVAL, "session: NULL buffer");
    if (!(flags & FNT_SUBMIT_HOST) && (!aligned(in, 4) || !aligned(out, 8)))
        return fail(FNT_E_INVAL, "session: misaligned device buffer");
    if (flags & ~FNT_SUBMIT_HOST) return fail(FNT_E_INVAL, "session: unknown flags 0x%x", flags);
    if ((flags & FNT_SUBMIT_HOST) && ((staging_bytes(n) + 255) & ~255ull) > s->pool.size()) {
        s->st.rejected++;
        return fail(FNT_E_BUSY, "session: request of %llu instants exceeds the staging pool",
                    (unsigned long long)n);
    }
    if (s->fatal) return check_fatal(s);
    Request r;
    r.ticket = s->next_ticket++;
    r.ch = ch;
    r.flags = flags;
    if (flags & FNT_SUBMIT_HOST) {
        r.host_in = in;
        r.host_out = out;
    } else {
        r.in = in;
        r.out = out;
    }
    r.n = n;
    r.blocks = n / 32;
    r.arrival_ns = arrival_ns ? arrival_ns : now_ns();
    Channel &c = s->chans[ch];
    c.queue.push_back(r.ticket);
    s->reqs.emplace(r.ticket, r);
    if (!c.in_rr) {
        c.in_rr = true;
        s->rr.push_back(ch);
    }
    s->st.submitted++;
    if (ticket) *ticket = r.ticket;
    s->cv_work.notify_all();
    return FNT_OK;
}

int fnt_session_submit(fnt_session *s, uint32_t ch, const int8_t *in, uint64_t n, int16_t *out,
                       uint32_t flags, uint64_t arrival_ns, uint64_t *ticket) {
    if (!s) return fail(FNT_E_INVAL, "session: NULL");
    std::lock_guard<std::mutex> g(s->mu);
    return submit_locked(s, ch, in, n, out, flags, arrival_ns, ticket);
}

int fnt_session_replay(fnt_session *s, const fnt_request *reqs, size_t nreq, uint64_t *tickets) {
    if (!s || (nreq && !reqs)) return fail(FNT_E_INVAL, "session replay: NULL");
    const uint64_t t0 = now_ns();
    for (size_t i = 0; i < nreq; ++i) {
        const uint64_t due = t0 + reqs[i].at_ns;
        while (now_ns() < due) {
            if (due - now_ns() > 200000) std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        std::lock_guard<std::mutex> g(s->mu);
        uint64_t tk = 0;
        int rc = submit_locked(s, reqs[i].ch, reqs[i].in, reqs[i].n, reqs[i].out, reqs[i].flags, due, &tk);
        if (rc) return rc;
        if (tickets) tickets[i] = tk;
    }
    return FNT_OK;
}

int fnt_session_poll(fnt_session *s, uint64_t ticket, int *done) {
    if (!s || !done) return fail(FNT_E_INVAL, "session: NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(FNT_E_STATE, "session: unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second.status == DONE || it->second.status == CANCELLED;
    return check_fatal(s);
}

int fnt_session_wait(fnt_session *s, uint64_t ticket) {
    if (!s) return fail(FNT_E_INVAL, "session: NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(FNT_E_STATE, "session: unknown ticket %llu", (unsigned long long)ticket);
        if (it->second.status == DONE || it->second.status == CANCELLED) return check_fatal(s);
        if (s->fatal) return check_fatal(s);
        s->cv_done.wait_for(lk, std::chrono::milliseconds(10));
    }
}

int fnt_session_drain(fnt_session *s) {
    if (!s) return fail(FNT_E_INVAL, "session: NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool pending = false;
        for (auto &kv : s->reqs)
            if (kv.second.status == QUEUED || kv.second.status == ACTIVE) {
                pending = true;
                break;
            }
        if (!pending && s->inflight.empty()) return check_fatal(s);
        if (s->fatal) return check_fatal(s);
        s->cv_done.wait_for(lk, std::chrono::milliseconds(10));
    }
}

int fnt_session_cancel(fnt_session *s, uint64_t ticket) {
    if (!s) return fail(FNT_E_INVAL, "session: NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(FNT_E_STATE, "session: unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.status != QUEUED) return fail(FNT_E_STATE, "session: ticket %llu already started", (unsigned long long)ticket);
    it->second.status = CANCELLED;
    s->st.cancelled++;
    s->cv_done.notify_all();
    return FNT_OK;
}

int fnt_session_get_state(fnt_session *s, uint32_t ch, void *host_buf, size_t *size) {
    if (!s || !size) return fail(FNT_E_INVAL, "session: NULL");
    if (!host_buf || *size < FNT_STATE_BYTES) {
        *size = FNT_STATE_BYTES;
        return host_buf ? fail(FNT_E_INVAL, "session: state buffer too small") : FNT_OK;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (ch >= s->cfg.max_channels || !s->chans[ch].registered)
        return fail(FNT_E_STATE, "session: channel %u not registered", ch);
    if (!channel_idle(s, ch)) return fail(FNT_E_STATE, "session: channel %u busy", ch);
    int rc = wait_channel_ticks(s, lk, ch);
    if (rc) return rc;
    const uint64_t pos = s->chans[ch].position;
    const int sel = s->chans[ch].tail_sel;
    lk.unlock();
    DevState h;
    hipError_t e = hipMemcpy(&h, s->dstate + ch, sizeof h, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sel)   // the current AEQ history is in the second copy
        e = hipMemcpy(h.aeq_tail, s->aeq_tail_alt + (uint64_t)ch * 64, 64, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "session: read state");
    h.position = pos;
    std::memcpy(host_buf, &h, sizeof h);
    *size = FNT_STATE_BYTES;
    return FNT_OK;
}

int fnt_session_set_state(fnt_session *s, uint32_t ch, const void *host_buf, size_t size) {
    if (!s || !host_buf) return fail(FNT_E_INVAL, "session: NULL");
    if (size != FNT_STATE_BYTES) return fail(FNT_E_INVAL, "session: state size %zu", size);
    DevState h;
    std::memcpy(&h, host_buf, sizeof h);
    for (int i = 0; i < 256; ++i)
        if (h.taps[i] < -8192 || h.taps[i] > 8191) return fail(FNT_E_RANGE, "session: state tap %d", i);
    for (int i = 0; i < 128; ++i)
        if (h.cdc_tail[i] < -16 || h.cdc_tail[i] > 15) return fail(FNT_E_RANGE, "session: state cdc tail");
    for (int i = 0; i < 64; ++i)
        if (h.aeq_tail[i] < -16 || h.aeq_tail[i] > 15) return fail(FNT_E_RANGE, "session: state aeq tail");
    std::unique_lock<std::mutex> lk(s->mu);
    if (ch >= s->cfg.max_channels || !s->chans[ch].registered)
        return fail(FNT_E_STATE, "session: channel %u not registered", ch);
    if (!channel_idle(s, ch)) return fail(FNT_E_STATE, "session: channel %u busy", ch);
    int rc = wait_channel_ticks(s, lk, ch);
    if (rc) return rc;
    s->chans[ch].position = h.position;
    s->chans[ch].tail_sel = 0;         // the imported history goes to DevState::aeq_tail
    lk.unlock();
    hipError_t e = hipMemcpy(s->dstate + ch, &h, sizeof h, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "session: write state");
    return FNT_OK;
}

int fnt_session_get_stats(fnt_session *s, fnt_session_stats *out) {
    if (!s || !out) return fail(FNT_E_INVAL, "session: NULL");
    std::lock_guard<std::mutex> g(s->mu);
    fnt_session_stats st = s->st;
    std::vector<double> v = s->lat_us;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto q = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
        st.p50_us = q(0.50);
        st.p99_us = q(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        st.mean_us = sum / v.size();
        st.max_us = v.back();
    }
    if (s->first_arrival != UINT64_MAX && s->last_completion > s->first_arrival) {
        st.first_arrival_s = s->first_arrival / 1e9;
        st.last_completion_s = s->last_completion / 1e9;
        st.gsamples_per_s = (double)st.instants_done / ((s->last_completion - s->first_arrival) / 1e9) / 1e9;
    }
    *out = st;
    return FNT_OK;
}

int fnt_session_destroy(fnt_session *s) {
    if (!s) return FNT_OK;
    int rc = fnt_session_drain(s);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
        s->cv_inflight.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    if (s->compl_.joinable()) s->compl_.join();
    (void)hipStreamSynchronize(s->copy_in);
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->copy_out);
    free_session(s);
    return rc;
}

}  // extern "C"
