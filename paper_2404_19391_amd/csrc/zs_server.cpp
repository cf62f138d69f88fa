// zs_server.cpp - request loop of the codec on one GPU.
//
// Resident compressed shards share one dictionary; random-access decompression
// requests (line ids of a shard) and compression requests (new lines) arrive
// from any host thread.  A scheduler thread admits them into a fixed number of
// slots, one HIP stream each, so that the work of many requests overlaps on
// the device.  A request is admitted by its device footprint, which is exact:
// a first stage runs the call in size-only mode (output offsets only), and the
// output buffer is taken from the device arena only once its size is known.
// Device and pinned host memory come from two arenas made at creation, so the
// loop itself never calls hipMalloc.  Stages end with events that the
// scheduler polls; results are copied to pinned host memory and handed to the
// waiting caller.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/zsmiles.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one block of memory (offsets), 256-byte granules.
class Arena {
  public:
    void init(uint8_t* base, uint64_t size) {
        base_ = base;
        size_ = size;
        free_.clear();
        free_[0] = size;
        used_ = 0;
    }
    uint8_t* alloc(uint64_t bytes) {
        bytes = (bytes + 255) & ~(uint64_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                sizes_[off] = bytes;
                used_ += bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(uint8_t* p) {
        if (!p) return;
        const uint64_t off = (uint64_t)(p - base_);
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        uint64_t len = s->second;
        sizes_.erase(s);
        used_ -= len;
        uint64_t start = off;
        // merge with the free block before and the one after
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        auto nx = free_.find(start + len);
        if (nx != free_.end()) {
            len += nx->second;
            free_.erase(nx);
        }
        free_[start] = len;
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

  private:
    uint8_t* base_ = nullptr;
    uint64_t size_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
    std::unordered_map<uint64_t, uint64_t> sizes_;
};

enum Kind { kDecompress = 1, kCompress = 2 };
enum Stage { kQueued, kSizing, kRunning, kDone };

struct Request {
    uint64_t ticket;
    Kind kind;
    uint32_t shard;
    uint32_t flags;
    uint64_t n;          // ids or lines
    uint64_t in_bytes;   // compression input bytes
    Stage stage = kQueued;
    int slot = -1;
    // host inputs, copied at submission into pinned memory
    uint8_t* h_in = nullptr;    // ids (n * 8) or lines (in_bytes) + offsets (n + 1) * 8
    uint64_t h_in_size = 0;
    // device buffers
    uint8_t* d_in = nullptr;    // ids, or lines then offsets
    uint64_t* d_off = nullptr;  // output offsets (n + 1)
    uint8_t* d_ws = nullptr;
    uint64_t ws_bytes = 0;
    zs_result* d_res = nullptr;
    uint8_t* d_out = nullptr;
    uint64_t total = 0;
    uint64_t opt_cap = 0;  // compression: output bytes reserved before the size is known
    // host outputs (pinned)
    uint8_t* h_out = nullptr;   // result word, offsets, bytes
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t footprint = 0;
    int32_t fail = 0;  // a launch or copy failed (zs_status); the request ends with it
};

// Record the first failure of a request's stage.
inline void note(Request* r, int32_t st) {
    if (st != ZS_OK && r->fail == 0) r->fail = st;
}
inline void note_hip(Request* r, hipError_t e) {
    if (e != hipSuccess) note(r, ZS_EDEVICE);
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    Request* req = nullptr;
};

struct Shard {
    const uint8_t* in;
    uint64_t in_bytes;
    const uint64_t* off;
    uint64_t n;
};

}  // namespace

struct zs_server {
    const zs_dict* dict = nullptr;
    int device = 0;
    uint8_t* d_base = nullptr;
    uint8_t* h_base = nullptr;
    Arena dev, host;
    std::vector<Slot> slots;
    std::vector<Shard> shards;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    zs_server_stats stats{};
};

namespace {

uint64_t a256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// Output bytes a compression request reserves before its size is known: its
// input size plus a newline per line holds any line that does not grow
// (every SMILES-alphabet line with the default dictionary); a larger output
// ends the first call with ZS_ENOSPC and complete offsets, and the request is
// run again with an output of the exact size.
uint64_t optimistic_cap(const Request* r) { return r->in_bytes + r->n; }

// Device bytes a request needs before its output size is known.
uint64_t stage1_bytes(const Request* r) {
    uint64_t b = a256((r->n + 1) * 8) + a256(sizeof(zs_result)) + a256(r->ws_bytes);
    if (r->kind == kDecompress) b += a256(r->n * 8);
    else b += a256(r->in_bytes + 16) + a256((r->n + 1) * 8) + a256(optimistic_cap(r) + 16);
    return b;
}

void free_device(zs_server* s, Request* r) {
    s->dev.release(r->d_in);
    s->dev.release((uint8_t*)r->d_off);
    s->dev.release(r->d_ws);
    s->dev.release((uint8_t*)r->d_res);
    s->dev.release(r->d_out);
    r->d_in = r->d_ws = r->d_out = nullptr;
    r->d_off = nullptr;
    r->d_res = nullptr;
}

// Stage 1: inputs to the device and the size-only call; the output size
// comes back with the event.  Returns false if the arenas are full.
bool start_sizing(zs_server* s, Slot& sl, Request* r) {
    const uint64_t need = stage1_bytes(r);
    if (s->dev.size() - s->dev.used() < need) return false;
    r->d_off = (uint64_t*)s->dev.alloc((r->n + 1) * 8);
    r->d_res = (zs_result*)s->dev.alloc(sizeof(zs_result));
    r->d_ws = s->dev.alloc(r->ws_bytes);
    r->d_in = s->dev.alloc(r->kind == kDecompress ? r->n * 8 : a256(r->in_bytes + 16) + (r->n + 1) * 8);
    if (r->kind == kCompress) {
        r->opt_cap = optimistic_cap(r);
        r->d_out = s->dev.alloc(r->opt_cap + 16);
    }
    uint8_t* hres = s->host.alloc(64);
    if (!r->d_off || !r->d_res || !r->d_ws || !r->d_in || !hres || (r->kind == kCompress && !r->d_out)) {
        free_device(s, r);
        s->host.release(hres);
        return false;
    }
    r->h_out = hres;
    hipStream_t st = sl.stream;
    memset(r->h_out, 0, 8);
    note_hip(r, hipMemcpyAsync(r->d_in, r->h_in, r->h_in_size, hipMemcpyHostToDevice, st));
    if (r->kind == kDecompress) {
        const Shard& sh = s->shards[r->shard];
        note(r, zs_decompress_lines(s->dict, sh.in, sh.in_bytes, sh.off, sh.n, (const uint64_t*)r->d_in, r->n,
                                    nullptr, 0, r->d_off, r->d_ws, r->ws_bytes, r->d_res, st));
    } else {
        // compression runs at once into the reserved output; the offsets are
        // complete even when the output does not fit
        const uint64_t* doff = (const uint64_t*)(r->d_in + a256(r->in_bytes + 16));
        note(r, zs_compress(s->dict, r->d_in, r->in_bytes, doff, r->n, r->d_out, r->opt_cap, r->d_off, r->flags,
                            r->d_ws, r->ws_bytes, r->d_res, st));
    }
    if (!r->fail) note_hip(r, hipMemcpyAsync(r->h_out, r->d_off + r->n, 8, hipMemcpyDeviceToHost, st));
    if (!r->fail) note_hip(r, hipMemcpyAsync(r->h_out + 16, r->d_res, sizeof(zs_result), hipMemcpyDeviceToHost, st));
    note_hip(r, hipEventRecord(sl.ev, st));
    r->stage = kSizing;
    r->slot = (int)(&sl - s->slots.data());
    r->t_admit = now_s();
    sl.req = r;
    return true;
}

// Stage 2: the output buffer of the exact size, the call, the copies back; a
// compression whose output fitted the reserved buffer only copies back.
// Returns false (and waits) if the arenas cannot hold the output yet.
bool start_running(zs_server* s, Slot& sl, Request* r) {
    memcpy(&r->total, r->h_out, 8);
    if (r->fail) r->total = 0;
    if (r->kind == kCompress && !r->fail) {
        zs_result first;
        memcpy(&first, r->h_out + 16, sizeof first);
        if (first.code != ZS_ENOSPC && r->total <= r->opt_cap) {
            const uint64_t hb = 64 + a256((r->n + 1) * 8) + r->total + 16;
            uint8_t* hout = s->host.alloc(hb);
            if (!hout) return false;
            s->host.release(r->h_out);
            r->h_out = hout;
            r->footprint = stage1_bytes(r);
            hipStream_t st = sl.stream;
            memset(r->h_out, 0, 64);
            note_hip(r, hipMemcpyAsync(r->h_out, r->d_res, sizeof(zs_result), hipMemcpyDeviceToHost, st));
            note_hip(r, hipMemcpyAsync(r->h_out + 64, r->d_off, (r->n + 1) * 8, hipMemcpyDeviceToHost, st));
            if (r->total)
                note_hip(r, hipMemcpyAsync(r->h_out + 64 + a256((r->n + 1) * 8), r->d_out, r->total,
                                           hipMemcpyDeviceToHost, st));
            note_hip(r, hipEventRecord(sl.ev, st));
            r->stage = kRunning;
            return true;
        }
        // larger than reserved: give the reservation back and run again at the exact size
        s->dev.release(r->d_out);
        r->d_out = nullptr;
    }
    uint8_t* dout = s->dev.alloc(r->total + 16);
    const uint64_t hb = 64 + a256((r->n + 1) * 8) + r->total + 16;
    uint8_t* hout = s->host.alloc(hb);
    if (!dout || !hout) {
        s->dev.release(dout);
        s->host.release(hout);
        return false;
    }
    s->host.release(r->h_out);
    r->h_out = hout;
    r->d_out = dout;
    r->footprint = stage1_bytes(r) + a256(r->total + 16);
    hipStream_t st = sl.stream;
    memset(r->h_out, 0, 64);
    if (!r->fail) {
        if (r->kind == kDecompress) {
            const Shard& sh = s->shards[r->shard];
            note(r, zs_decompress_lines(s->dict, sh.in, sh.in_bytes, sh.off, sh.n, (const uint64_t*)r->d_in, r->n,
                                        r->d_out, r->total + 16, r->d_off, r->d_ws, r->ws_bytes, r->d_res, st));
        } else {
            const uint64_t* doff = (const uint64_t*)(r->d_in + a256(r->in_bytes + 16));
            note(r, zs_compress(s->dict, r->d_in, r->in_bytes, doff, r->n, r->d_out, r->total + 16, r->d_off,
                                r->flags, r->d_ws, r->ws_bytes, r->d_res, st));
        }
    }
    if (!r->fail) {
        note_hip(r, hipMemcpyAsync(r->h_out, r->d_res, sizeof(zs_result), hipMemcpyDeviceToHost, st));
        note_hip(r, hipMemcpyAsync(r->h_out + 64, r->d_off, (r->n + 1) * 8, hipMemcpyDeviceToHost, st));
        if (r->total)
            note_hip(r, hipMemcpyAsync(r->h_out + 64 + a256((r->n + 1) * 8), r->d_out, r->total,
                                       hipMemcpyDeviceToHost, st));
    }
    note_hip(r, hipEventRecord(sl.ev, st));
    r->stage = kRunning;
    return true;
}

// True if the request's output can never be held, even by arenas that hold
// nothing else: the device arena must take its stage-1 buffers plus the
// output, the host arena its pinned input plus the reply (offsets, bytes).
bool never_fits(const zs_server* s, const Request* r) {
    const uint64_t dev_need = stage1_bytes(r) + a256(r->total + 16);
    const uint64_t host_need = a256(r->h_in_size + 16) + a256(64 + a256((r->n + 1) * 8) + r->total + 16) + 256;
    return dev_need > s->dev.size() || host_need > s->host.size();
}

// End a request that failed before its output was written (reply: the code,
// no offsets, no bytes).
void finish_failed(zs_server* s, Slot& sl, Request* r, int32_t code) {
    note(r, code);
    r->total = 0;
    free_device(s, r);
    s->host.release(r->h_in);
    r->h_in = nullptr;
    r->stage = kDone;
    r->t_done = now_s();
    r->slot = -1;
    sl.req = nullptr;
    s->stats.completed++;
    s->stats.busy_s += r->t_done - r->t_admit;
    s->cv_done.notify_all();
}

void run_loop(zs_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool busy = false, progressed = false;
        // advance the slots whose stage has finished
        for (Slot& sl : s->slots) {
            Request* r = sl.req;
            if (!r) continue;
            busy = true;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            note_hip(r, q);
            if (r->stage == kSizing) {
                if (start_running(s, sl, r)) {
                    progressed = true;
                } else if (never_fits(s, r)) {
                    // requeueing it would size it again forever
                    finish_failed(s, sl, r, ZS_ENOSPC);
                    progressed = true;
                } else {
                    // no room for the output: if no running request will free memory,
                    // give this one's memory back and queue it again at the front
                    bool running = false;
                    for (const Slot& o : s->slots) running |= o.req && o.req->stage == kRunning;
                    if (!running) {
                        free_device(s, r);
                        s->host.release(r->h_out);
                        r->h_out = nullptr;
                        r->stage = kQueued;
                        r->slot = -1;
                        sl.req = nullptr;
                        s->queue.push_front(r);
                        s->stats.deferred++;
                        progressed = true;
                    }
                }
            } else if (r->stage == kRunning) {
                r->stage = kDone;
                r->t_done = now_s();
                free_device(s, r);
                s->host.release(r->h_in);
                r->h_in = nullptr;
                sl.req = nullptr;
                s->stats.completed++;
                s->stats.busy_s += r->t_done - r->t_admit;
                progressed = true;
                s->cv_done.notify_all();
            }
        }
        // admit queued requests into free slots, in arrival order
        for (Slot& sl : s->slots) {
            if (sl.req || s->queue.empty()) continue;
            Request* r = s->queue.front();
            if (!start_sizing(s, sl, r)) {
                s->stats.deferred++;
                break;  // not enough memory now: keep the order, try after a completion
            }
            s->queue.pop_front();
            s->stats.admitted++;
            busy = true;
            progressed = true;
        }
        const uint64_t used = s->dev.used();
        if (used > s->stats.peak_device_bytes) s->stats.peak_device_bytes = used;
        if (s->stop && s->queue.empty() && !busy) break;
        if (!busy && s->queue.empty()) {
            s->cv_work.wait(lk);
        } else if (!progressed) {
            // device work in flight: poll again shortly
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

zs_status zs_server_create(const zs_dict* d, const zs_server_config* cfg, zs_server** out) {
    if (!d || !cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->device_bytes < (1u << 20) ||
        cfg->host_bytes < (1u << 20))
        return ZS_EINVAL;
    zs_server* s = new (std::nothrow) zs_server;
    if (!s) return ZS_ENOMEM;
    s->dict = d;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return ZS_EDEVICE;
    }
    if (hipMalloc(&s->d_base, cfg->device_bytes) != hipSuccess) {
        delete s;
        return ZS_ENOMEM;
    }
    if (hipHostMalloc(&s->h_base, cfg->host_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(s->d_base);
        delete s;
        return ZS_ENOMEM;
    }
    s->dev.init(s->d_base, cfg->device_bytes);
    s->host.init(s->h_base, cfg->host_bytes);
    s->slots.resize(cfg->slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            zs_server_destroy(s);
            return ZS_EDEVICE;
        }
    }
    s->worker = std::thread(run_loop, s);
    *out = s;
    return ZS_OK;
}

zs_status zs_server_add_shard(zs_server* s, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                              uint64_t n_lines, uint32_t* shard) {
    if (!s || !in_off || !shard || (!in && in_bytes)) return ZS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    s->shards.push_back(Shard{in, in_bytes, in_off, n_lines});
    *shard = (uint32_t)(s->shards.size() - 1);
    return ZS_OK;
}

static zs_status submit(zs_server* s, Request* r, uint64_t* ticket) {
    std::lock_guard<std::mutex> g(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = now_s();
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    s->stats.submitted++;
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return ZS_OK;
}

// Pinned copy of the caller's input, made on the calling thread; waits for
// room in the host arena.
static uint8_t* host_copy(zs_server* s, const void* a, uint64_t na, const void* b, uint64_t nb) {
    std::unique_lock<std::mutex> lk(s->mu);
    uint8_t* p = nullptr;
    while (!(p = s->host.alloc(a256(na + 16) + nb))) {
        if (s->host.used() == 0) return nullptr;  // can never fit
        s->cv_done.wait(lk);
    }
    lk.unlock();
    if (na) memcpy(p, a, na);
    if (nb) memcpy(p + a256(na + 16), b, nb);
    return p;
}

zs_status zs_server_submit_decompress(zs_server* s, uint32_t shard, const uint64_t* ids, uint64_t n_ids,
                                      uint64_t* ticket) {
    if (!s || !ticket || (!ids && n_ids) || n_ids == 0) return ZS_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (shard >= s->shards.size()) return ZS_EINVAL;
    }
    Request* r = new (std::nothrow) Request;
    if (!r) return ZS_ENOMEM;
    r->kind = kDecompress;
    r->shard = shard;
    r->n = n_ids;
    r->ws_bytes = zs_workspace_bytes(ZS_OP_DECOMPRESS_LINES, n_ids);
    if (stage1_bytes(r) + a256(n_ids * 8) > s->dev.size()) {
        delete r;
        return ZS_ENOSPC;
    }
    r->h_in = host_copy(s, ids, n_ids * 8, nullptr, 0);
    r->h_in_size = n_ids * 8;
    if (!r->h_in) {
        delete r;
        return ZS_ENOSPC;
    }
    return submit(s, r, ticket);
}

zs_status zs_server_submit_compress(zs_server* s, const uint8_t* lines, uint64_t bytes, const uint64_t* off,
                                    uint64_t n_lines, uint32_t flags, uint64_t* ticket) {
    if (!s || !ticket || !off || (!lines && bytes) || n_lines == 0 || (flags & ~ZS_F_PREPROCESS)) return ZS_EINVAL;
    Request* r = new (std::nothrow) Request;
    if (!r) return ZS_ENOMEM;
    r->kind = kCompress;
    r->n = n_lines;
    r->in_bytes = bytes;
    r->flags = flags;
    r->ws_bytes = zs_workspace_bytes(ZS_OP_COMPRESS, n_lines);
    if (stage1_bytes(r) > s->dev.size()) {
        delete r;
        return ZS_ENOSPC;
    }
    // lines, then offsets at a 256-byte boundary past them (the device copy keeps the layout)
    r->h_in = host_copy(s, lines, bytes, off, (n_lines + 1) * 8);
    r->h_in_size = a256(bytes + 16) + (n_lines + 1) * 8;
    if (!r->h_in) {
        delete r;
        return ZS_ENOSPC;
    }
    return submit(s, r, ticket);
}

zs_status zs_server_wait(zs_server* s, uint64_t ticket, zs_reply* out) {
    if (!s || !out) return ZS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return ZS_EINVAL;
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->stage == kDone; });
    zs_result res;
    memcpy(&res, r->h_out, sizeof res);
    out->code = r->fail ? r->fail : res.code;
    out->first_bad = r->fail ? -1 : res.first_bad;
    out->n = r->n;
    out->off = r->fail ? nullptr : (const uint64_t*)(r->h_out + 64);
    out->data = r->fail ? nullptr : r->h_out + 64 + a256((r->n + 1) * 8);
    out->bytes = r->fail ? 0 : r->total;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    out->footprint = r->footprint;
    return ZS_OK;
}

void zs_server_release(zs_server* s, uint64_t ticket) {
    if (!s) return;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->stage != kDone) return;
    s->host.release(it->second->h_out);
    delete it->second;
    s->reqs.erase(it);
    s->cv_done.notify_all();
}

zs_status zs_server_get_stats(zs_server* s, zs_server_stats* out) {
    if (!s || !out) return ZS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->device_bytes_in_use = s->dev.used();
    return ZS_OK;
}

void zs_server_destroy(zs_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : s->reqs) delete kv.second;
    if (s->d_base) (void)hipFree(s->d_base);
    if (s->h_base) (void)hipHostFree(s->h_base);
    delete s;
}

}  // extern "C"
