// Native served form: continuous batching of circular convolutions behind the
// C ABI (ntt_server_*).  Host code only: the arithmetic runs in conv_batched.
//
// A request's life (device arenas): submit copies f and g into a pinned staging
// block (rows f, g, h) and queues the request; the scheduler thread admits
// queued requests in arrival order into slots of a buddy allocator over three
// device arenas, uploads each batch's rows, runs one conv_batched over the
// batch on the next stream, downloads the results into the staging blocks and
// records an event; when the event has passed, the slots are freed and waiters
// are woken; wait copies the result out and returns the staging block to the
// pool.
//
// Host arenas (ntt_server_create_host): the slot is taken at submission, in
// three pinned host arenas (chunks of 2^arena_log2 words, a new chunk when the
// others are full) that the device reads and writes directly; submit copies f
// and g into the slot, a batch is requests of one chunk and one conv_batched
// call whose kernels load f, g and store h there (no copies), and wait copies
// the result out and frees the slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/nttmi.h"

namespace nttmi {
ntt_status reserve_stream(void* stream, size_t bytes);   // api.cpp
void release_stream_caches(void* stream);             // api.cpp
}

namespace {

using Clock = std::chrono::steady_clock;

// Power-of-two buddy allocator over [0, 2^top) words: alloc(k) gives a free
// block of 2^k words aligned to 2^k (lowest address first), free merges buddies.
class Buddy {
  public:
    explicit Buddy(int top) : top_(top), free_(top + 1) { free_[top].insert(0); }
    bool alloc(int k, uint64_t* off) {
        if (k > top_) return false;
        int j = k;
        while (j <= top_ && free_[j].empty()) ++j;
        if (j > top_) return false;
        uint64_t o = *free_[j].begin();
        free_[j].erase(free_[j].begin());
        while (j > k) {   // split, keep the lower half
            --j;
            free_[j].insert(o + (1ull << j));
        }
        *off = o;
        return true;
    }
    void release(uint64_t o, int k) {
        while (k < top_) {
            const uint64_t b = o ^ (1ull << k);
            auto it = free_[k].find(b);
            if (it == free_[k].end()) break;
            free_[k].erase(it);
            o = std::min(o, b);
            ++k;
        }
        free_[k].insert(o);
    }

  private:
    int top_;
    std::vector<std::set<uint64_t>> free_;
};

// Pinned host blocks by exact size, reused.
class PinnedPool {
  public:
    void* get(size_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        auto& v = free_[bytes];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        all_.push_back(p);
        return p;
    }
    void put(void* p, size_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        free_[bytes].push_back(p);
    }
    ~PinnedPool() {
        for (void* p : all_) (void)hipHostFree(p);
    }

  private:
    std::mutex mu_;
    std::map<size_t, std::vector<void*>> free_;
    std::vector<void*> all_;
};

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3, Q_STAGED = 4 };

// Host arenas: three pinned arenas of 2^top words, read and written by the
// batch kernels at the addresses the device sees (dF, dG, dH).
struct Chunk {
    char *F = nullptr, *G = nullptr, *H = nullptr;
    void *dF = nullptr, *dG = nullptr, *dH = nullptr;
    Buddy buddy{0};
};

struct Req {
    uint64_t id = 0;
    uint32_t log2n = 0;
    uint64_t off = 0;
    Chunk* chunk = nullptr;    // host arenas: the chunk holding the slot
    char* staging = nullptr;   // device arenas: f, g, h rows of 2^log2n words
    size_t staging_bytes = 0;
    Clock::time_point arrival;
    int state = Q_QUEUED;
    bool waiting = false;   // a thread is in ntt_server_wait on this ticket
};

struct Batch {
    std::vector<Req*> reqs;
    hipEvent_t ev = nullptr;
};

}  // namespace

struct ntt_server {
    uint64_t m = 0, root = 0;
    uint32_t rlo = 0, bits = 0, arena_log2 = 0;
    uint32_t max_batch = 1, max_inflight = 1;
    uint64_t max_batch_elems = 0;
    // requests of 2^solo_log2n words and more run as batches of their own (0:
    // never).  In a batch with other items a long convolution runs on one
    // workgroup and every request of the batch completes with it; alone it
    // takes the four-step form spread over the chip.
    uint32_t solo_log2n = 16;
    // how often the scheduler polls the events of batches in flight (tuning
    // override: NTTMI_SERVER_POLL_US)
    int poll_us = 10;
    size_t wb = 4;
    int dev = 0;
    bool host = false;                 // host arenas (ntt_server_create_host)
    std::vector<Chunk*> chunks;        // host arenas, guarded by mu
    char *F = nullptr, *G = nullptr, *H = nullptr;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    // completed batches' events, reused by later batches (touched by the
    // scheduler thread only, and by destroy after it has stopped)
    std::vector<hipEvent_t> free_events;
    Buddy buddy{0};
    PinnedPool pool;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req*> queue;
    std::vector<Batch> inflight;
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th;

    // statistics: the latencies of the last LAT_WINDOW completed requests (a
    // ring, so that a long-running server holds a bounded amount)
    static constexpr size_t LAT_WINDOW = size_t(1) << 20;
    std::vector<double> lat_ms;
    size_t lat_next = 0;
    uint64_t completed = 0, batches = 0, batched_reqs = 0;
    void record_latency(double ms) {
        if (lat_ms.size() < LAT_WINDOW) lat_ms.push_back(ms);
        else lat_ms[lat_next] = ms;
        lat_next = (lat_next + 1) % LAT_WINDOW;
        completed += 1;
    }

    void run();
    bool launch(std::vector<Req*>& adm);
    Chunk* host_slot(uint32_t log2n, uint64_t* off, std::unique_lock<std::mutex>& lk);
};

// Host arenas: a slot of 2^log2n words in the first chunk with room, else in a
// new chunk; null when pinned memory runs out.  Called with mu held through
// `lk`, which it releases while it allocates a chunk (milliseconds), so that
// the scheduler thread and the other clients do not wait for that; chunks are
// kept until the server is destroyed.
Chunk* ntt_server::host_slot(uint32_t log2n, uint64_t* off, std::unique_lock<std::mutex>& lk) {
    for (Chunk* c : chunks)
        if (c->buddy.alloc((int)log2n, off)) return c;
    const size_t bytes = (size_t(1) << arena_log2) * wb;
    lk.unlock();
    Chunk* c = new Chunk();
    c->buddy = Buddy((int)arena_log2);
    hipError_t e = hipHostMalloc((void**)&c->F, bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->G, bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->H, bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->dF, c->F, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->dG, c->G, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->dH, c->H, 0);
    if (e != hipSuccess || !c->buddy.alloc((int)log2n, off)) {
        for (char* p : {c->F, c->G, c->H})
            if (p) (void)hipHostFree(p);
        delete c;
        lk.lock();
        return nullptr;
    }
    lk.lock();
    chunks.push_back(c);
    return c;
}

// Uploads, convolves and downloads one admitted batch; false if a HIP call or
// conv_batched failed (nothing of the batch is then in flight).
bool ntt_server::launch(std::vector<Req*>& adm) {
    hipStream_t s = streams[next_stream++ % streams.size()];
    std::vector<uint8_t> lg(adm.size());
    std::vector<uint64_t> off(adm.size());
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < adm.size() && host; ++i) {
        lg[i] = (uint8_t)adm[i]->log2n;
        off[i] = adm[i]->off;
    }
    for (size_t i = 0; i < adm.size() && e == hipSuccess && !host; ++i) {
        Req* r = adm[i];
        const size_t row = (size_t(1) << r->log2n) * wb;
        lg[i] = (uint8_t)r->log2n;
        off[i] = r->off;
        e = hipMemcpyAsync(F + r->off * wb, r->staging, row, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(G + r->off * wb, r->staging + row, row, hipMemcpyHostToDevice, s);
    }
    ntt_batch_desc d{(uint32_t)adm.size(), lg.data(), off.data()};
    // host arenas: one chunk per batch (admission keeps it so)
    const void* bF = host ? adm[0]->chunk->dF : (const void*)F;
    const void* bG = host ? adm[0]->chunk->dG : (const void*)G;
    void* bH = host ? adm[0]->chunk->dH : (void*)H;
    if (e != hipSuccess || conv_batched(m, root, rlo, bits, &d, bF, bG, bH, NTT_FLAG_TRANSIENT, s) != NTT_OK) {
        // copies already enqueued may still run: let them finish before the
        // caller frees the slots
        (void)hipStreamSynchronize(s);
        return false;
    }
    for (size_t i = 0; i < adm.size() && e == hipSuccess && !host; ++i) {
        Req* r = adm[i];
        const size_t row = (size_t(1) << r->log2n) * wb;
        e = hipMemcpyAsync(r->staging + 2 * row, H + r->off * wb, row, hipMemcpyDeviceToHost, s);
    }
    Batch b;
    if (e == hipSuccess) {
        if (!free_events.empty()) {
            b.ev = free_events.back();
            free_events.pop_back();
        } else {
            e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(b.ev, s);
    if (e != hipSuccess) {
        // the stream may still run what was enqueued: let it finish first
        (void)hipStreamSynchronize(s);
        if (b.ev) (void)hipEventDestroy(b.ev);
        return false;
    }
    b.reqs = adm;
    std::lock_guard<std::mutex> g(mu);
    inflight.push_back(std::move(b));
    batches += 1;
    batched_reqs += adm.size();
    return true;
}

void ntt_server::run() {
    (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (stop && queue.empty() && inflight.empty()) break;
        // admit in arrival order while slots are free
        std::vector<Req*> adm;
        uint64_t elems = 0;
        if (inflight.size() < max_inflight) {
            while (!queue.empty() && adm.size() < max_batch) {
                Req* r = queue.front();
                const uint64_t size = 1ull << r->log2n;
                const bool solo = solo_log2n != 0 && r->log2n >= solo_log2n;
                if (!adm.empty() && (solo || elems + size > max_batch_elems)) break;
                if (host) {
                    if (!adm.empty() && r->chunk != adm[0]->chunk) break;
                } else {
                    uint64_t o = 0;
                    if (!buddy.alloc((int)r->log2n, &o)) break;
                    r->off = o;
                }
                queue.pop_front();
                r->state = Q_RUNNING;
                elems += size;
                adm.push_back(r);
                if (solo) break;
            }
        }
        bool progress = false;
        if (!adm.empty()) {
            lk.unlock();
            const bool ok = launch(adm);
            lk.lock();
            if (!ok) {
                for (Req* r : adm) {
                    if (!host) buddy.release(r->off, (int)r->log2n);
                    r->state = Q_FAILED;
                }
                cv_done.notify_all();
            }
            progress = true;
        }
        // retire finished batches
        for (size_t i = 0; i < inflight.size();) {
            const hipError_t q = hipEventQuery(inflight[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            const auto now = Clock::now();
            for (Req* r : inflight[i].reqs) {
                if (!host) buddy.release(r->off, (int)r->log2n);   // host arenas: freed by wait
                r->state = q == hipSuccess ? Q_DONE : Q_FAILED;
                if (q == hipSuccess) record_latency(std::chrono::duration<double, std::milli>(now - r->arrival).count());
            }
            if (q == hipSuccess) free_events.push_back(inflight[i].ev);
            else (void)hipEventDestroy(inflight[i].ev);
            inflight.erase(inflight.begin() + (long)i);
            progress = true;
        }
        if (progress) {
            cv_done.notify_all();
            continue;
        }
        // nothing launched or retired: sleep until a submission, or poll the
        // batches in flight again shortly
        cv_sched.wait_for(lk, std::chrono::microseconds(inflight.empty() ? 2000 : poll_us));
    }
}

namespace {

// ntt_server_create / ntt_server_create_host: device or host arenas.
ntt_status create_server(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits, uint32_t arena_log2,
                         uint32_t streams, uint32_t max_batch, uint64_t max_batch_elems, uint32_t max_inflight,
                         bool host, ntt_server** out) {
    if (!out) return NTT_E_ARG;
    *out = nullptr;
    if (arena_log2 > 28 || streams < 1 || streams > 16 || max_batch < 1 || max_inflight < 1) return NTT_E_ARG;
    // modulus, word width and root, as conv_batched checks them (an empty batch)
    uint8_t lg0 = 0;
    uint64_t off0 = 0;
    ntt_batch_desc d0{0, &lg0, &off0};
    int dummy = 0;
    ntt_status st = conv_batched(m, root, root_log2order, elem_bits, &d0, &dummy, &dummy, &dummy, 0, nullptr);
    if (st != NTT_OK) return st;
    ntt_server* s = new ntt_server();
    s->m = m;
    s->root = root;
    s->rlo = root_log2order;
    s->bits = elem_bits;
    s->wb = elem_bits / 8;
    s->arena_log2 = arena_log2;
    s->max_batch = max_batch;
    s->max_inflight = max_inflight;
    s->max_batch_elems = max_batch_elems ? max_batch_elems : (1ull << arena_log2);
    s->buddy = Buddy((int)arena_log2);
    s->host = host;
    if (const char* pe = std::getenv("NTTMI_SERVER_POLL_US")) {
        const int v = std::atoi(pe);
        if (v > 0 && v <= 10000) s->poll_us = v;
    }
    hipError_t e = hipGetDevice(&s->dev);
    const size_t bytes = (size_t(1) << arena_log2) * s->wb;
    if (e == hipSuccess && !host) e = hipMalloc((void**)&s->F, bytes);
    if (e == hipSuccess && !host) e = hipMalloc((void**)&s->G, bytes);
    if (e == hipSuccess && !host) e = hipMalloc((void**)&s->H, bytes);
    // the largest scratch a batch launch takes: at most two resident
    // workgroups per CU, 2N words each for N up to the arena, and never more
    // than 1 GiB; reserved with each stream's work queue now rather than on
    // the request path
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->dev);
    const size_t reserve = std::min<size_t>(size_t(1) << 30, size_t(2) * (size_t)std::max(cus, 1) * bytes * 2);
    for (uint32_t i = 0; i < streams && e == hipSuccess; ++i) {
        hipStream_t h = nullptr;
        e = hipStreamCreateWithFlags(&h, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(h);
        if (e == hipSuccess && nttmi::reserve_stream(h, reserve) != NTT_OK) e = hipErrorOutOfMemory;
    }
    if (e != hipSuccess) {
        for (hipStream_t h : s->streams) {
            nttmi::release_stream_caches(h);
            (void)hipStreamDestroy(h);
        }
        if (s->F) (void)hipFree(s->F);
        if (s->G) (void)hipFree(s->G);
        if (s->H) (void)hipFree(s->H);
        delete s;
        return (e == hipErrorOutOfMemory) ? NTT_E_NOMEM : NTT_E_DEVICE;
    }
    s->th = std::thread([s] { s->run(); });
    *out = s;
    return NTT_OK;
}

}  // namespace

extern "C" {

ntt_status ntt_server_create(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                             uint32_t arena_log2, uint32_t streams, uint32_t max_batch, uint64_t max_batch_elems,
                             uint32_t max_inflight, ntt_server** out) {
    return create_server(m, root, root_log2order, elem_bits, arena_log2, streams, max_batch, max_batch_elems,
                         max_inflight, false, out);
}

ntt_status ntt_server_create_host(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                                  uint32_t arena_log2, uint32_t streams, uint32_t max_batch,
                                  uint64_t max_batch_elems, uint32_t max_inflight, ntt_server** out) {
    return create_server(m, root, root_log2order, elem_bits, arena_log2, streams, max_batch, max_batch_elems,
                         max_inflight, true, out);
}

ntt_status ntt_server_submit(ntt_server* s, const void* f, const void* g, uint32_t log2n, uint64_t* ticket) {
    if (!s || !f || !g || !ticket) return NTT_E_ARG;
    if (log2n > s->rlo || log2n > s->arena_log2) return NTT_E_LENGTH;
    const auto arrival = Clock::now();
    const size_t row = (size_t(1) << log2n) * s->wb;
    if (s->host) {
        // the slot first (under the lock), the copies outside it, then queued
        Req* r = new Req();
        r->log2n = log2n;
        r->state = Q_STAGED;
        char *fp = nullptr, *gp = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            Chunk* c = s->stop ? nullptr : s->host_slot(log2n, &r->off, lk);
            if (!c) {
                const bool stopped = s->stop;
                delete r;
                return stopped ? NTT_E_ARG : NTT_E_NOMEM;
            }
            r->chunk = c;
            r->id = s->next_id++;
            s->reqs[r->id] = r;
            fp = c->F + r->off * s->wb;
            gp = c->G + r->off * s->wb;
        }
        std::memcpy(fp, f, row);
        std::memcpy(gp, g, row);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->arrival = arrival;
            r->state = Q_QUEUED;
            s->queue.push_back(r);
            *ticket = r->id;
        }
        s->cv_sched.notify_one();
        return NTT_OK;
    }
    char* st = (char*)s->pool.get(3 * row);
    if (!st) return NTT_E_NOMEM;
    std::memcpy(st, f, row);
    std::memcpy(st + row, g, row);
    Req* r = new Req();
    r->log2n = log2n;
    r->staging = st;
    r->staging_bytes = 3 * row;
    r->arrival = arrival;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            s->pool.put(st, 3 * row);
            delete r;
            return NTT_E_ARG;
        }
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->queue.push_back(r);
        *ticket = r->id;
    }
    s->cv_sched.notify_one();
    return NTT_OK;
}

ntt_status ntt_server_stage(ntt_server* s, uint32_t log2n, void** f, void** g, uint64_t* ticket) {
    if (!s || !f || !g || !ticket) return NTT_E_ARG;
    if (log2n > s->rlo || log2n > s->arena_log2) return NTT_E_LENGTH;
    const size_t row = (size_t(1) << log2n) * s->wb;
    if (s->host) {
        Req* r = new Req();
        r->log2n = log2n;
        r->state = Q_STAGED;
        std::unique_lock<std::mutex> lk(s->mu);
        Chunk* c = s->stop ? nullptr : s->host_slot(log2n, &r->off, lk);
        if (!c) {
            const bool stopped = s->stop;
            delete r;
            return stopped ? NTT_E_ARG : NTT_E_NOMEM;
        }
        r->chunk = c;
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        *ticket = r->id;
        *f = c->F + r->off * s->wb;
        *g = c->G + r->off * s->wb;
        return NTT_OK;
    }
    char* st = (char*)s->pool.get(3 * row);
    if (!st) return NTT_E_NOMEM;
    Req* r = new Req();
    r->log2n = log2n;
    r->staging = st;
    r->staging_bytes = 3 * row;
    r->state = Q_STAGED;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        s->pool.put(st, 3 * row);
        delete r;
        return NTT_E_ARG;
    }
    r->id = s->next_id++;
    s->reqs[r->id] = r;
    *ticket = r->id;
    *f = st;
    *g = st + row;
    return NTT_OK;
}

ntt_status ntt_server_submit_staged(ntt_server* s, uint64_t ticket) {
    if (!s) return NTT_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second->state != Q_STAGED || s->stop) return NTT_E_ARG;
        Req* r = it->second;
        r->arrival = Clock::now();
        r->state = Q_QUEUED;
        s->queue.push_back(r);
    }
    s->cv_sched.notify_one();
    return NTT_OK;
}

ntt_status ntt_server_wait(ntt_server* s, uint64_t ticket, void* h, double timeout_s) {
    if (!s || !h) return NTT_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return NTT_E_ARG;
    Req* r = it->second;
    // never queued, or a second waiter (the first releases the request, which
    // the second would then read)
    if (r->state == Q_STAGED || r->waiting) return NTT_E_ARG;
    r->waiting = true;
    auto ready = [r] { return r->state == Q_DONE || r->state == Q_FAILED; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        r->waiting = false;
        return NTT_E_TIMEOUT;
    }
    s->reqs.erase(it);
    lk.unlock();
    const size_t row = (size_t(1) << r->log2n) * s->wb;
    const bool ok = r->state == Q_DONE;
    if (s->host) {
        if (ok) std::memcpy(h, r->chunk->H + r->off * s->wb, row);
        lk.lock();
        r->chunk->buddy.release(r->off, (int)r->log2n);
        lk.unlock();
    } else {
        if (ok) std::memcpy(h, r->staging + 2 * row, row);
        s->pool.put(r->staging, r->staging_bytes);
    }
    delete r;
    return ok ? NTT_OK : NTT_E_DEVICE;
}

ntt_status ntt_server_stats(ntt_server* s, uint64_t* completed, double* mean_batch, double* p50_ms, double* p99_ms,
                            uint32_t reset) {
    if (!s) return NTT_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v(s->lat_ms);
    std::sort(v.begin(), v.end());
    auto pct = [&v](double q) {
        if (v.empty()) return 0.0;
        const double x = q * (double)(v.size() - 1);   // linear interpolation between order statistics
        const size_t i = (size_t)x;
        const double fr = x - (double)i;
        return i + 1 < v.size() ? v[i] * (1 - fr) + v[i + 1] * fr : v[i];
    };
    if (completed) *completed = s->completed;
    if (mean_batch) *mean_batch = s->batches ? (double)s->batched_reqs / (double)s->batches : 0.0;
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (reset) {
        s->lat_ms.clear();
        s->lat_next = 0;
        s->completed = 0;
        s->batches = 0;
        s->batched_reqs = 0;
    }
    return NTT_OK;
}

ntt_status ntt_server_set_solo(ntt_server* s, uint32_t solo_log2n) {
    if (!s) return NTT_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->solo_log2n = solo_log2n;
    return NTT_OK;
}

void ntt_server_destroy(ntt_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->th.joinable()) s->th.join();   // the thread drains the queue and the batches in flight first
    for (auto& kv : s->reqs) {
        if (!s->host) s->pool.put(kv.second->staging, kv.second->staging_bytes);
        delete kv.second;
    }
    for (Chunk* c : s->chunks) {
        for (char* p : {c->F, c->G, c->H}) (void)hipHostFree(p);
        delete c;
    }
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    for (hipStream_t h : s->streams) {
        nttmi::release_stream_caches(h);
        (void)hipStreamDestroy(h);
    }
    if (s->F) (void)hipFree(s->F);
    if (s->G) (void)hipFree(s->G);
    if (s->H) (void)hipFree(s->H);
    delete s;
}

}  // extern "C"
