// C-ABI of the library: validation, plan and workspace caches, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/nttmi.h"
#include "launch.hpp"
#include "numtheory.hpp"

using namespace nttmi;

namespace {

struct Plan {
    DevPlan dev{};
    double2* dP = nullptr;
    double* dTT = nullptr;
    uint32_t* dTT32 = nullptr;
};

struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool keep = false;   // descriptor cache: referenced by a captured graph, never evicted
    uint32_t pins = 0;   // descriptor cache: looked up by calls whose kernels are not yet enqueued
};

// Cumulative launch and upload counts by form (ntt_launch_counts).
std::atomic<uint64_t> g_counts[NTT_COUNT_SLOTS];
inline void count(int k, uint64_t by = 1) { g_counts[k].fetch_add(by, std::memory_order_relaxed); }

// How conv_batched runs a batch: one persistent launch for the lengths it
// covers (multi) or one launch per length, and the form of each length's
// launch (ClassForm).  Chosen by the autotuner and cached per batch shape.
enum ClassForm : uint8_t {
    CF_DEFAULT = 0,      // LDS kernel of 256 threads / persistent fused kernel at full occupancy
    CF_SMALL_WAVE = 1,   // LDS kernel with one wave per workgroup
    CF_FUSED_ONE = 2,    // persistent fused kernel, one workgroup per CU
    CF_FOURSTEP = 3,     // unfused four-step: column, row and column launches over all items,
                         // 512-thread blocks
    CF_FOURSTEP_256 = 4, // the same with 256-thread blocks (twice the workgroups per phase)
};
struct BatchForm {
    bool multi = false;
    std::map<uint32_t, uint8_t> cls;   // log2n -> ClassForm
};

// Staging ring of transient descriptors on one stream.  Slot k owns a pinned
// host buffer that the kernels read directly, at the address the device sees
// (no copy to device memory: one transfer engine operation less per call).
// Each upload first records, on the stream, the release event of the slot
// handed out before it: that event completes once everything enqueued so far,
// the kernels that read that slot included, has run.  A slot is refilled only
// after its release event has completed, so it is never overwritten while a
// kernel may still read it.
constexpr int RING_SLOTS = 8;
struct RingSlot {
    void* dev = nullptr;    // the device's address of `host`
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t rel = nullptr;
    bool recorded = false;
};
struct Ring {
    std::mutex mu;   // serialises uploads on the stream (the cache lock is not held while waiting)
    RingSlot slot[RING_SLOTS];
    unsigned next = 0;
    int last = -1;   // slot handed out by the previous upload
};

// Key of the descriptor cache, (device, content), and a comparator that also
// takes a view of a caller's vector, so that a lookup copies nothing.
using OffKey = std::pair<int, std::vector<uint64_t>>;
struct OffKeyView {
    int dev;
    const std::vector<uint64_t>* v;
};
struct OffKeyLess {
    using is_transparent = void;
    static bool lt(int da, const std::vector<uint64_t>& a, int db, const std::vector<uint64_t>& b) {
        return da != db ? da < db : a < b;
    }
    bool operator()(const OffKey& a, const OffKey& b) const { return lt(a.first, a.second, b.first, b.second); }
    bool operator()(const OffKey& a, const OffKeyView& b) const { return lt(a.first, a.second, b.dev, *b.v); }
    bool operator()(const OffKeyView& a, const OffKey& b) const { return lt(a.dev, *a.v, b.first, b.second); }
};

struct Caches {
    std::mutex mu;
    std::map<std::tuple<int, uint64_t, int, uint64_t>, Plan> plans;   // (dev, m, log2n, root)
    std::map<std::pair<int, void*>, Buf> work;                        // (dev, stream) -> scratch
    std::map<std::pair<int, void*>, Buf> flag;                        // (dev, stream) -> range flag
    std::map<std::pair<int, void*>, Buf> queue;                       // (dev, stream) -> work queue
    std::map<std::pair<int, void*>, Buf> tune;                        // (dev, stream) -> autotuning output
    std::map<std::vector<uint64_t>, struct BatchForm> forms;          // batch shape -> tuned form
    std::map<OffKey, Buf, OffKeyLess> offsets;                          // (dev, offsets) -> device copy
    std::map<std::pair<int, void*>, struct Ring> rings;               // (dev, stream) -> transient uploads
    std::vector<void*> retired;                                       // outgrown device buffers
    std::vector<void*> retired_host;                                  // outgrown pinned staging
    std::map<uint64_t, std::pair<int, int>> moduli;                   // m -> (log2 nu or -1, v2(m-1) or -1)
    std::map<int, int> cu_count;                                      // dev -> CUs
};

Caches& caches() {
    static Caches* c = new Caches();  // intentionally never destroyed
    return *c;
}

ntt_status hip_status(hipError_t e) {
    if (e == hipSuccess) return NTT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return NTT_E_NOMEM;
    return NTT_E_DEVICE;
}

// (log2 nu, v2) of a modulus: log2 of the order of 2 when m is prime and that
// order is a power of two (2 is a lambda-root of m: Sec. II, Prop. 2), and the
// 2-adic valuation of m - 1 when m is prime (the longest power-of-two length
// of the Euler form, Sec. I, Eq. 6); -1 where they do not apply.  Cached.
std::pair<int, int> modulus_info(uint64_t m) {
    Caches& c = caches();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.moduli.find(m);
        if (it != c.moduli.end()) return it->second;
    }
    int lnu = -1, v2 = -1;
    if (m >= 3 && is_prime64(m)) {
        lnu = log2_order_of_two(m);
        v2 = 0;
        while (((m - 1) >> v2 & 1) == 0) ++v2;
    }
    std::lock_guard<std::mutex> g(c.mu);
    c.moduli[m] = std::make_pair(lnu, v2);
    return std::make_pair(lnu, v2);
}

int modulus_log2nu(uint64_t m) { return modulus_info(m).first; }

// Checks m and the word width.  Default: the paper's moduli, primes of which 2
// is a lambda-root; *lnu = log2 nu bounds the length.  With NTT_FLAG_EULER any
// prime; *lnu = v2(m - 1) bounds the length.
ntt_status check_modulus_info(uint64_t m, uint32_t elem_bits, const std::pair<int, int>& info, int* lnu,
                              uint32_t flags) {
    *lnu = (flags & NTT_FLAG_EULER) ? info.second : info.first;
    if (*lnu < 0) return NTT_E_MODULUS;
    if (elem_bits == 32 && m >= (1ull << 24)) return NTT_E_MODULUS;
    if (elem_bits == 64 && m >= (1ull << 62)) return NTT_E_MODULUS;
    // 64-bit words: residues are carried exactly in fp64; the bounds of the
    // double-product reduction close (pass outputs <= 11 m, products exact)
    // for m < 2^46
    if (elem_bits == 64 && m >= (1ull << 46)) return NTT_E_UNSUPPORTED;
    return NTT_OK;
}

ntt_status check_modulus(uint64_t m, uint32_t elem_bits, int* lnu, uint32_t flags = 0) {
    if (elem_bits != 32 && elem_bits != 64) return NTT_E_ARG;
    return check_modulus_info(m, elem_bits, modulus_info(m), lnu, flags);
}

// root has exact order 2^k modulo m
bool root_has_order(uint64_t root, uint32_t k, uint64_t m) {
    const uint64_t r = root % m;
    if (k == 0) return r == 1;
    return powmod64(r, 1ull << (k - 1), m) == m - 1;
}

ntt_status validate(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, int* lnu, uint32_t flags) {
    ntt_status st = check_modulus(m, elem_bits, lnu, flags);
    if (st != NTT_OK) return st;
    if ((int)log2n > *lnu) return NTT_E_LENGTH;
    if (!root_has_order(root, log2n, m)) return NTT_E_ROOT;
    if (log2n > (uint32_t)MAX_LOG2N) return NTT_E_UNSUPPORTED;
    return NTT_OK;
}

template <class T>
hipError_t upload(T** d, const std::vector<T>& h) {
    hipError_t e = hipMalloc((void**)d, h.size() * sizeof(T));
    if (e != hipSuccess) {
        *d = nullptr;
        return e;
    }
    e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    // complete before any stream may read it (the copy runs on the null stream)
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    return e;
}

// Device tables of the plan (m, N = 2^log2n, root): the powers root^e mod m,
// e < N, which are the harmonics of the digital circle (Eq. 5) generated one
// factor at a time, and for four-step lengths the twiddles root^(+-t1 u2).
ntt_status get_plan(uint64_t m, uint32_t log2n, uint64_t root, int lnu, const Plan** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NTT_E_DEVICE;
    const uint64_t r = root % m;
    // log2 of the order of 2 (or -1), looked up before the cache lock is taken:
    // modulus_info takes the same (non-recursive) lock
    const int l2 = modulus_log2nu(m);
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    auto key = std::make_tuple(dev, m, (int)log2n, r);
    auto it = c.plans.find(key);
    if (it != c.plans.end()) {
        *out = &it->second;
        return NTT_OK;
    }
    const uint64_t N = 1ull << log2n;
    std::vector<double2> hP(N);
    uint64_t x = 1 % m;
    for (uint64_t e = 0; e < N; ++e) {
        hP[e] = tw_pair(x, m);
        x = mulmod64(x, r, m);
    }
    Plan p;
    hipError_t he = upload(&p.dP, hP);
    if (he == hipSuccess && (int)log2n > SMALL_MAX_LOG2N) {
        const int la = fs_la((int)log2n), lb = (int)log2n - la;
        const uint64_t A = 1ull << la, B = 1ull << lb;
        std::vector<double> tt(N);
        for (uint64_t u2 = 0; u2 < B; ++u2)
            for (uint64_t t1 = 0; t1 < A; ++t1) tt[u2 * A + t1] = hP[(t1 * u2) & (N - 1)].x;
        he = upload(&p.dTT, tt);
        if (he == hipSuccess && m < (1ull << 32)) {
            std::vector<uint32_t> t32(N);
            for (uint64_t e = 0; e < N; ++e) t32[e] = (uint32_t)tt[e];
            he = upload(&p.dTT32, t32);
        }
    }
    if (he != hipSuccess) {
        if (p.dP) (void)hipFree(p.dP);
        if (p.dTT) (void)hipFree(p.dTT);
        if (p.dTT32) (void)hipFree(p.dTT32);
        return hip_status(he);
    }
    // N^-1 mod m, the multiplicative inverse of N (Appendix A): 2^(nu - n)
    // when 2 has order nu = 2^lnu, else N^(m - 2) (Fermat, m prime)
    const uint64_t ninv = (l2 >= (int)log2n) ? powmod64(2, (1ull << l2) - log2n, m)
                                             : powmod64((1ull << log2n) % m, m - 2, m);
    (void)lnu;
    p.dev.P = p.dP;
    p.dev.TT = p.dTT;
    p.dev.TT32 = p.dTT32;
    p.dev.M = make_modc(m);
    p.dev.ninv = (double)ninv;
    p.dev.ninvq = (double)ninv / (double)m;
    p.dev.logn = (int)log2n;
    p.dev.nmask = (int)(N - 1);
    auto ins = c.plans.emplace(key, p);
    *out = &ins.first->second;
    return NTT_OK;
}

// The cached plan of (m, N, root) on the current device, or null; allocates
// nothing (no insertion into any cache).
const Plan* find_plan(uint64_t m, uint32_t log2n, uint64_t root) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.plans.find(std::make_tuple(dev, m, (int)log2n, root % m));
    return it == c.plans.end() ? nullptr : &it->second;
}

// (log2 nu, v2) of m if cached, without computing or inserting it.
bool modulus_info_cached(uint64_t m, std::pair<int, int>* out) {
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.moduli.find(m);
    if (it == c.moduli.end()) return false;
    *out = it->second;
    return true;
}

// Per-(device, stream) buffer of at least `bytes`.  Growing it first waits for
// the stream, so no enqueued kernel still uses the old buffer.
ntt_status get_buf(std::map<std::pair<int, void*>, Buf>& pool, void* stream, size_t bytes, void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NTT_E_DEVICE;
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    Buf& b = pool[std::make_pair(dev, stream)];
    if (b.bytes < bytes) {
        // at least double, so that the retired buffers sum to less than the
        // live one
        const size_t cap = std::max(bytes, 2 * b.bytes);
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess) return hip_status(e);
        // the old buffer is retired, not freed: work enqueued earlier and
        // graphs captured earlier keep using it (freed by ntt_release_caches)
        if (b.ptr) c.retired.push_back(b.ptr);
        b.ptr = p;
        b.bytes = cap;
    }
    *out = b.ptr;
    return NTT_OK;
}

// Per-(device, stream) work queue of the persistent kernels: two uint32 words,
// zeroed once here, on the stream itself so that the first kernel is ordered
// after the zeroing (a plain hipMemset runs on the null stream, which does not
// order the non-blocking streams callers use); every launch leaves them zero
// again.  Creation is refused while the stream is being captured.  Only the
// persistent forms (k_conv_fused, k_conv_multi) create it, so a call made
// before a capture prepares the queue only if it takes one of those forms:
// the same batch shape on the same stream does.
ntt_status get_queue(void* stream, uint32_t** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NTT_E_DEVICE;
    std::lock_guard<std::mutex> g(caches().mu);
    Buf& b = caches().queue[std::make_pair(dev, stream)];
    if (!b.ptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
            return NTT_E_DEVICE;
        hipError_t e = hipMalloc(&b.ptr, 256);
        if (e == hipSuccess) e = hipMemsetAsync(b.ptr, 0, 256, (hipStream_t)stream);
        if (e != hipSuccess) {
            if (b.ptr) (void)hipFree(b.ptr);
            b.ptr = nullptr;
            return hip_status(e);
        }
        b.bytes = 256;
        count(NTT_COUNT_QUEUE_CREATED);
    }
    *out = (uint32_t*)b.ptr;
    return NTT_OK;
}

// A descriptor in device memory for one call.  When it comes from the
// content-addressed cache it stays pinned there, so that no eviction frees it,
// until the call has enqueued the kernel that reads it (end of scope).
using OffMap = std::map<OffKey, Buf, OffKeyLess>;
struct DescRef {
    const uint64_t* ptr = nullptr;
    bool pinned = false;
    OffMap::iterator it;
    DescRef() = default;
    DescRef(const DescRef&) = delete;
    DescRef& operator=(const DescRef&) = delete;
    ~DescRef();
};

// Device copy of an offsets array, cached by content (uploaded once) and
// pinned in `ref` for the caller.  A full cache (256 entries) first waits for
// the device and frees every entry that no call holds pinned and no captured
// graph references: kernels enqueued earlier have then run, and descriptors
// looked up but not yet launched (by this or another thread) are pinned.
ntt_status get_offsets(const std::vector<uint64_t>& h, DescRef* ref, bool keep = false) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NTT_E_DEVICE;
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.offsets.find(OffKeyView{dev, &h});
    if (it == c.offsets.end()) {
        if (c.offsets.size() >= 256) {
            (void)hipDeviceSynchronize();
            for (auto e = c.offsets.begin(); e != c.offsets.end();) {
                if (e->second.keep || e->second.pins) {
                    ++e;
                } else {
                    (void)hipFree(e->second.ptr);
                    e = c.offsets.erase(e);
                    count(NTT_COUNT_DESC_EVICTED);
                }
            }
        }
        Buf b;
        hipError_t e = hipMalloc(&b.ptr, h.size() * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMemcpy(b.ptr, h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);   // complete before any stream reads it
        if (e != hipSuccess) {
            if (b.ptr) (void)hipFree(b.ptr);
            return hip_status(e);
        }
        b.bytes = h.size() * sizeof(uint64_t);
        it = c.offsets.emplace(OffKey(dev, h), b).first;
        count(NTT_COUNT_DESC_CACHED);
    }
    if (keep) it->second.keep = true;
    it->second.pins += 1;
    ref->ptr = (const uint64_t*)it->second.ptr;
    ref->pinned = true;
    ref->it = it;
    return NTT_OK;
}

DescRef::~DescRef() {
    if (!pinned) return;
    std::lock_guard<std::mutex> g(caches().mu);
    it->second.pins -= 1;
}

// Device copy of a descriptor used by one call: through the stream's staging
// ring when `transient` and the stream is not being captured, else through the
// content-addressed cache above (entries looked up under capture are kept for
// the life of the caches).
ntt_status stream_capturing(void* stream, bool* capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) return NTT_E_DEVICE;
    *capturing = cs != hipStreamCaptureStatusNone;
    return NTT_OK;
}

ntt_status get_desc(const std::vector<uint64_t>& h, bool transient, void* stream, DescRef* out) {
    bool capturing = false;
    if (stream_capturing(stream, &capturing) != NTT_OK) return NTT_E_DEVICE;
    if (!transient || capturing) return get_offsets(h, out, capturing);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NTT_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = std::max<size_t>(8, h.size() * sizeof(uint64_t));
    Caches& c = caches();
    Ring* rp = nullptr;
    {
        std::lock_guard<std::mutex> g(c.mu);
        rp = &c.rings[std::make_pair(dev, stream)];   // map nodes stay put
    }
    Ring& r = *rp;
    std::lock_guard<std::mutex> g(r.mu);
    hipError_t e = hipSuccess;
    if (r.last >= 0) {
        // the previous upload's kernels are enqueued by now
        RingSlot& prev = r.slot[r.last];
        e = hipEventRecord(prev.rel, s);
        if (e != hipSuccess) return hip_status(e);
        prev.recorded = true;
    }
    const int k = (int)(r.next++ % RING_SLOTS);
    RingSlot& sl = r.slot[k];
    if (!sl.rel) e = hipEventCreateWithFlags(&sl.rel, hipEventDisableTiming);
    else if (sl.recorded) e = hipEventSynchronize(sl.rel);   // its last readers have run
    if (e != hipSuccess) return hip_status(e);
    sl.recorded = false;
    r.last = k;
    if (sl.cap < bytes) {
        // at least double; the outgrown buffers are retired, not freed (a free
        // would wait for the whole device)
        const size_t cap = std::max<size_t>({bytes, 2 * sl.cap, 65536});
        void *d = nullptr, *hh = nullptr;
        e = hipHostMalloc(&hh, cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostGetDevicePointer(&d, hh, 0);
        if (e != hipSuccess) {
            if (hh) (void)hipHostFree(hh);
            return hip_status(e);
        }
        if (sl.host) {
            std::lock_guard<std::mutex> gc(c.mu);
            c.retired_host.push_back(sl.host);
        }
        sl.dev = d;
        sl.host = hh;
        sl.cap = cap;
    }
    std::memcpy(sl.host, h.data(), h.size() * sizeof(uint64_t));
    out->ptr = (const uint64_t*)sl.dev;
    count(NTT_COUNT_DESC_RING);
    return NTT_OK;
}

int cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Caches& c = caches();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.cu_count.find(dev);
        if (it != c.cu_count.end()) return it->second;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
    std::lock_guard<std::mutex> g(c.mu);
    c.cu_count[dev] = n;
    return n;
}

// [a, a+na) and [b, b+nb) in bytes: 0 disjoint, 1 identical start and size, 2 partial
int overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    if (x + na <= y || y + nb <= x) return 0;
    if (x == y && na == nb) return 1;
    return 2;
}

ntt_status check_range(uint32_t wbits, const void* x, uint64_t n, uint64_t m, void* stream) {
    void* flag = nullptr;
    ntt_status st = get_buf(caches().flag, stream, sizeof(uint32_t), &flag);
    if (st != NTT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_range_check((int)wbits, x, n, m, (uint32_t*)flag, s);
    uint32_t hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e);
    return hflag ? NTT_E_RANGE : NTT_OK;
}

// One convolution of length 2^log2n (plan already built) on the stream.
ntt_status conv_one(const Plan* p, uint32_t wbits, uint32_t log2n, const void* f, const void* g, void* h,
                    void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if ((int)log2n <= SMALL_MAX_LOG2N) {
        count(NTT_COUNT_SMALL);
        return hip_status(launch_conv_small((int)wbits, log2n, f, g, h, nullptr, 1, p->dev, s));
    }
    void* ws = nullptr;
    ntt_status st = get_buf(caches().work, stream, ((size_t)2 * (wbits / 8)) << log2n, &ws);
    if (st != NTT_OK) return st;
    count(NTT_COUNT_FOURSTEP);
    return hip_status(launch_conv_fourstep((int)wbits, log2n, f, g, h, 1, 0, ws, p->dev, s, nullptr, (uint32_t)cu_count()));
}

// `batch` contiguous rows of N = 2^log2n, forward or inverse, plan built.  The
// four-step path runs in chunks of rows whose scratch stays within 1 GiB.
ntt_status ntt_rows(const Plan* p, uint32_t elem_bits, uint32_t log2n, bool inv, const void* x, void* X,
                    uint32_t batch, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    count(NTT_COUNT_TRANSFORM);
    if ((int)log2n <= SMALL_MAX_LOG2N)
        return hip_status(launch_ntt_small((int)elem_bits, log2n, inv, x, X, batch, p->dev, s));
    const size_t wb = elem_bits / 8;
    const uint64_t per = (uint64_t)wb << log2n;
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, (1ull << 30) / per), 65535);
    void* ws = nullptr;
    ntt_status st = get_buf(caches().work, stream, (size_t)(std::min(chunk, batch) * per), &ws);
    if (st != NTT_OK) return st;
    for (uint32_t r = 0; r < batch; r += chunk) {
        const uint32_t k = std::min(chunk, batch - r);
        const hipError_t e = launch_ntt_fourstep((int)elem_bits, log2n, inv, (const char*)x + (size_t)r * per,
                                                 (char*)X + (size_t)r * per, k, ws, p->dev, s, (uint32_t)cu_count());
        if (e != hipSuccess) return hip_status(e);
    }
    return NTT_OK;
}

ntt_status ntt_any(bool inv, uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* x, void* X,
                   uint32_t batch, uint32_t flags, void* stream) {
    int lnu = 0;
    ntt_status st = validate(m, log2n, root, elem_bits, &lnu, flags);
    if (st != NTT_OK) return st;
    if (batch == 0) return NTT_OK;
    if (!x || !X) return NTT_E_ARG;
    const size_t bytes = ((size_t)batch << log2n) * (elem_bits / 8);
    if (overlap(x, bytes, X, bytes) == 2) return NTT_E_ARG;
    if (flags & NTT_FLAG_CHECK_RANGE) {
        st = check_range(elem_bits, x, (uint64_t)batch << log2n, m, stream);
        if (st != NTT_OK) return st;
    }
    const Plan* p = nullptr;
    st = get_plan(m, log2n, root, lnu, &p);
    if (st != NTT_OK) return st;
    return ntt_rows(p, elem_bits, log2n, inv, x, X, batch, stream);
}

// One launch for the items of one length class: the LDS kernel below 2^13,
// the persistent fused four-step kernel above.
// c items of length 2^n: at offsets base + i 2^n (doffs null), else at the
// device offsets doffs[i] (base 0).
ntt_status launch_items(uint32_t n, uint32_t c, uint64_t base, const uint64_t* doffs, const Plan* p,
                        uint32_t elem_bits, const char* F, const char* G, char* H, hipStream_t s, void* stream,
                        uint8_t form) {
    const size_t wb = elem_bits / 8;
    const bool contiguous = doffs == nullptr;
    ntt_status st = NTT_OK;
    if ((int)n <= SMALL_MAX_LOG2N) {
        count(NTT_COUNT_SMALL);
        return hip_status(launch_conv_small((int)elem_bits, n, F + base * wb, G + base * wb, H + base * wb, doffs, c,
                                            p->dev, s, form == CF_SMALL_WAVE ? SMALL_TILE_WAVE : SMALL_TILE_256));
    }
    // multi-launch four-step form: every phase spreads all items over the
    // chip; scratch 2N words per item, within 1 GiB
    const bool fourstep_ok = contiguous && (((uint64_t)2 * c * wb) << n) <= (1ull << 30);
    // (workgroup size: by the default rule, or as the form names it)
    auto fourstep = [&]() -> ntt_status {
        void* ws = nullptr;
        const ntt_status e = get_buf(caches().work, stream, (size_t)(((uint64_t)2 * c * wb) << n), &ws);
        if (e != NTT_OK) return e;
        count(NTT_COUNT_FOURSTEP);
        const int tt = form == CF_FOURSTEP ? 512 : (form == CF_FOURSTEP_256 ? 256 : 0);
        return hip_status(launch_conv_fourstep((int)elem_bits, n, F + base * wb, G + base * wb, H + base * wb, c,
                                               1ull << n, ws, p->dev, s, nullptr, (uint32_t)cu_count(), tt));
    };
    if ((form == CF_FOURSTEP || form == CF_FOURSTEP_256) && fourstep_ok) return fourstep();
    // persistent fused form: grid = resident workgroups, bounded by a 1 GiB
    // scratch budget (2N words per workgroup)
    // tuning override: NTTMI_FUSED_WG_PER_CU caps resident workgroups per CU
    int per_cu = form == CF_FUSED_ONE ? 1 : std::max(1, fused_blocks_per_cu((int)elem_bits, n));
    if (const char* e = std::getenv("NTTMI_FUSED_WG_PER_CU")) {
        const int cap = std::atoi(e);
        if (cap > 0) per_cu = std::min(per_cu, cap);
    }
    uint64_t grid = (uint64_t)std::max(1, cu_count()) * per_cu;
    const uint64_t per_wg = ((uint64_t)2 * wb) << n;
    grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, (1ull << 30) / per_wg));
    // Fewer items than two thirds of the resident workgroups: the fused form,
    // one item per workgroup, would leave CUs idle, so the four-step form runs
    // (measured 1.1-2.4x faster there at 2^15..2^19; above it the fused form
    // is faster or equal)
    if (form == CF_DEFAULT && fourstep_ok && 3ull * c < 2ull * grid) return fourstep();
    grid = std::min<uint64_t>(grid, c);
    void* ws = nullptr;
    st = get_buf(caches().work, stream, (size_t)(grid * per_wg), &ws);
    if (st != NTT_OK) return st;
    uint32_t* q = nullptr;
    st = get_queue(stream, &q);
    if (st != NTT_OK) return st;
    count(NTT_COUNT_FUSED);
    return hip_status(launch_conv_fused((int)elem_bits, n, F + base * wb, G + base * wb, H + base * wb, doffs, c,
                                        ws, q, (uint32_t)grid, p->dev, s));
}

ntt_status launch_class(uint32_t n, const std::vector<uint64_t>& off, const Plan* p, uint32_t elem_bits,
                        const char* F, const char* G, char* H, hipStream_t s, void* stream,
                        uint8_t form = CF_DEFAULT, bool transient = false) {
    const uint32_t c = (uint32_t)off.size();
    // contiguous uniform run: offsets base + i N, no table needed
    bool contiguous = true;
    for (uint32_t i = 1; i < c && contiguous; ++i) contiguous = off[i] == off[0] + ((uint64_t)i << n);
    DescRef doffs;   // pinned until the launch below is enqueued
    if (!contiguous) {
        const ntt_status st = get_desc(off, transient, stream, &doffs);
        if (st != NTT_OK) return st;
    }
    return launch_items(n, c, contiguous ? off[0] : 0, doffs.ptr, p, elem_bits, F, G, H, s, stream, form);
}

// One persistent launch for every class of length <= 2^nmax.  The task list
// runs longest first (each four-step item is a task; shorter items go in tiles
// of multi_tile(n)), so the short tasks fill in behind the long ones.  The
// item offsets, the task list and the per-length plans are uploaded once per
// distinct batch and cached by content.
ntt_status launch_multi(const std::map<uint32_t, std::vector<uint64_t>>& cls,
                        std::map<uint32_t, const Plan*>& plans, uint32_t nmax, uint32_t elem_bits, const char* F,
                        const char* G, char* H, hipStream_t s, void* stream, bool transient = false) {
    // the upload: item offsets (task order), then two words per task (first
    // item; log2n | count << 32), then (transient) the plans; sized up front
    size_t nitems = 0, ntask_words = 0;
    for (auto& kv : cls) {
        if (kv.first > nmax) continue;
        const size_t tile = (int)kv.first <= SMALL_MAX_LOG2N ? (size_t)multi_tile((int)kv.first) : 1;
        nitems += kv.second.size();
        ntask_words += 2 * ((kv.second.size() + tile - 1) / tile);
    }
    std::vector<uint64_t> blob;
    blob.reserve(nitems + ntask_words + 2 + (nmax + 1) * sizeof(DevPlan) / 8);
    std::vector<uint64_t> tasks;
    tasks.reserve(ntask_words);
    uint32_t nbig = 0;
    for (auto it = cls.rbegin(); it != cls.rend(); ++it) {
        const uint32_t n = it->first;
        if (n > nmax) continue;
        const std::vector<uint64_t>& off = it->second;
        const uint32_t tile = (int)n <= SMALL_MAX_LOG2N ? (uint32_t)multi_tile((int)n) : 1u;
        if ((int)n > SMALL_MAX_LOG2N) nbig = std::max(nbig, n);
        const size_t first = blob.size();   // the class's items follow in task order
        for (size_t i = 0; i < off.size(); i += tile) {
            const uint32_t k = (uint32_t)std::min<size_t>(tile, off.size() - i);
            tasks.push_back(first + i);
            tasks.push_back((uint64_t)n | ((uint64_t)k << 32));
        }
        blob.insert(blob.end(), off.begin(), off.end());
    }
    const uint32_t ntasks = (uint32_t)(tasks.size() / 2);
    if (ntasks == 0) return NTT_OK;
    const size_t task_at = blob.size();
    blob.insert(blob.end(), tasks.begin(), tasks.end());
    // per-length plans, indexed by log2n
    static_assert(sizeof(DevPlan) % 8 == 0 && alignof(DevPlan) <= 16, "DevPlan is uploaded as 8-byte words");
    std::vector<DevPlan> hp(nmax + 1);
    std::memset((void*)hp.data(), 0, hp.size() * sizeof(DevPlan));
    for (auto& kv : plans)
        if (kv.first <= nmax) hp[kv.first] = kv.second->dev;
    std::vector<uint64_t> pw(hp.size() * sizeof(DevPlan) / 8);
    std::memcpy(pw.data(), hp.data(), pw.size() * 8);
    // one upload: items and tasks, padded to 16 bytes, then the plans (one
    // descriptor, pinned until the launch is enqueued)
    const size_t plans_at = (blob.size() + 1) & ~(size_t)1;
    blob.resize(plans_at, 0);
    blob.insert(blob.end(), pw.begin(), pw.end());
    DescRef desc;
    ntt_status st = get_desc(blob, transient, stream, &desc);
    if (st != NTT_OK) return st;
    const uint64_t* dblob = desc.ptr;
    const uint64_t* dplans = dblob + plans_at;
    const size_t wb = elem_bits / 8;
    const uint64_t scratch_words = nbig ? (2ull << nbig) : 1;
    uint64_t grid = (uint64_t)std::max(1, cu_count()) * std::max(1, multi_blocks_per_cu((int)elem_bits));
    grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, (1ull << 30) / (scratch_words * wb)));
    grid = std::min<uint64_t>(grid, ntasks);
    void* ws = nullptr;
    st = get_buf(caches().work, stream, (size_t)(grid * scratch_words * wb), &ws);
    if (st != NTT_OK) return st;
    uint32_t* q = nullptr;
    st = get_queue(stream, &q);
    if (st != NTT_OK) return st;
    count(NTT_COUNT_MULTI);
    return hip_status(launch_conv_multi((int)elem_bits, F, G, H, dblob + task_at, ntasks, dblob, ws, scratch_words, q,
                                        (uint32_t)grid, (const DevPlan*)(const void*)dplans, s));
}

// Runs a batch in the given form.
ntt_status run_batch(const BatchForm& form, const std::map<uint32_t, std::vector<uint64_t>>& cls,
                     std::map<uint32_t, const Plan*>& plans, uint32_t nmax, uint32_t elem_bits, const char* F,
                     const char* G, char* H, hipStream_t s, void* stream, bool transient = false) {
    ntt_status st = NTT_OK;
    if (form.multi) {
        st = launch_multi(cls, plans, nmax, elem_bits, F, G, H, s, stream, transient);
        if (st != NTT_OK) return st;
    }
    for (auto& kv : cls) {
        if (form.multi && kv.first <= nmax) continue;
        auto it = form.cls.find(kv.first);
        const uint8_t cf = it == form.cls.end() ? (uint8_t)CF_DEFAULT : it->second;
        st = launch_class(kv.first, kv.second, plans[kv.first], elem_bits, F, G, H, s, stream, cf, transient);
        if (st != NTT_OK) return st;
    }
    return NTT_OK;
}

// Batch shape: modulus, word width, and per length the item count rounded
// down to a power of two.
std::vector<uint64_t> shape_key(uint64_t m, uint32_t elem_bits, const std::map<uint32_t, std::vector<uint64_t>>& cls) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<uint64_t> k{(uint64_t)dev, m, elem_bits};
    for (auto& kv : cls) {
        uint64_t c = kv.second.size(), b = 0;
        while (c >>= 1) ++b;
        k.push_back(((uint64_t)kv.first << 32) | b);
    }
    return k;
}

std::vector<uint64_t> shape_key_uniform(uint64_t m, uint32_t elem_bits, uint32_t n, uint64_t count) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    uint64_t b = 0;
    while (count >>= 1) ++b;
    return {(uint64_t)dev, m, elem_bits, ((uint64_t)n << 32) | b};
}

bool lookup_form(const std::vector<uint64_t>& key, BatchForm* out) {
    std::lock_guard<std::mutex> g(caches().mu);
    auto it = caches().forms.find(key);
    if (it == caches().forms.end()) return false;
    *out = it->second;
    return true;
}

void store_form(const std::vector<uint64_t>& key, const BatchForm& f) {
    std::lock_guard<std::mutex> g(caches().mu);
    caches().forms[key] = f;
}

// Milliseconds of `run` on the stream: one untimed run, then the best of three.
template <class F>
ntt_status time_ms(hipStream_t s, F run, float* best) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return NTT_E_DEVICE;
    }
    ntt_status st = run();
    *best = 3.4e38f;
    for (int r = 0; st == NTT_OK && r < 3; ++r) {
        hipError_t e = hipEventRecord(a, s);
        if (e == hipSuccess) st = run();
        if (st == NTT_OK && e == hipSuccess) e = hipEventRecord(b, s);
        if (st == NTT_OK && e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (st == NTT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) st = hip_status(e);
        if (st == NTT_OK) *best = std::min(*best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

// The autotuner: times every candidate form of each length on this batch
// (each length alone), keeps the fastest, then times the single persistent
// launch against the sum of the per-length bests.  Trial outputs go to a
// scratch buffer when h overlaps f or g, so the operands survive; the caller
// then runs the chosen form once more for the result.
ntt_status autotune(const std::map<uint32_t, std::vector<uint64_t>>& cls, std::map<uint32_t, const Plan*>& plans,
                    uint32_t nmax, uint32_t elem_bits, const char* F, const char* G, char* H, uint64_t total,
                    hipStream_t s, void* stream, BatchForm* out) {
    const size_t wb = elem_bits / 8;
    const size_t bytes = (size_t)total * wb;
    char* T = H;
    if (overlap(F, bytes, H, bytes) || overlap(G, bytes, H, bytes)) {
        void* t = nullptr;
        ntt_status st = get_buf(caches().tune, stream, bytes, &t);
        if (st != NTT_OK) return st;
        T = (char*)t;
    }
    BatchForm best;
    float sum_covered = 0.f;
    for (auto& kv : cls) {
        const uint32_t n = kv.first;
        std::vector<uint8_t> cand{CF_DEFAULT};
        if ((int)n <= SMALL_MAX_LOG2N) {
            cand.push_back(CF_SMALL_WAVE);
        } else {
            if (fused_blocks_per_cu((int)elem_bits, n) > 1) cand.push_back(CF_FUSED_ONE);
            cand.push_back(CF_FOURSTEP);
            if (n <= FOURSTEP_256_MAX_LOG2N) cand.push_back(CF_FOURSTEP_256);
        }
        float tbest = 3.4e38f;
        uint8_t fbest = CF_DEFAULT;
        for (uint8_t cf : cand) {
            float ms = 0.f;
            ntt_status st = time_ms(s, [&] { return launch_class(n, kv.second, plans[n], elem_bits, F, G, T, s, stream, cf); },
                                    &ms);
            if (st != NTT_OK) return st;
            if (ms < tbest) {
                tbest = ms;
                fbest = cf;
            }
        }
        best.cls[n] = fbest;
        if (n <= nmax) sum_covered += tbest;
    }
    size_t covered = 0;
    for (auto& kv : cls) covered += kv.first <= nmax ? 1 : 0;
    best.multi = false;
    if (covered >= 2) {
        float ms = 0.f;
        ntt_status st = time_ms(s, [&] { return launch_multi(cls, plans, nmax, elem_bits, F, G, T, s, stream); }, &ms);
        if (st != NTT_OK) return st;
        best.multi = ms < sum_covered;
    }
    *out = best;
    return NTT_OK;
}

}  // namespace

namespace nttmi {

// Sizes the workspace of `stream` to at least `bytes` and creates its work
// queue now, so that later calls on the stream allocate nothing (for owners
// of long-lived streams, such as the native server).
ntt_status reserve_stream(void* stream, size_t bytes) {
    void* ws = nullptr;
    ntt_status st = get_buf(caches().work, stream, bytes, &ws);
    uint32_t* q = nullptr;
    if (st == NTT_OK) st = get_queue(stream, &q);
    return st;
}

// Drops the per-stream state of `stream` on the current device (workspace,
// flag, work queue, tuning buffer, descriptor ring) once the stream is idle;
// for owners of streams that are about to be destroyed.
void release_stream_caches(void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    (void)hipStreamSynchronize((hipStream_t)stream);
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    const auto key = std::make_pair(dev, stream);
    for (auto* pool : {&c.work, &c.flag, &c.queue, &c.tune}) {
        auto it = pool->find(key);
        if (it == pool->end()) continue;
        if (it->second.ptr) (void)hipFree(it->second.ptr);
        pool->erase(it);
    }
    auto r = c.rings.find(key);
    if (r != c.rings.end()) {
        for (RingSlot& sl : r->second.slot) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.rel) (void)hipEventDestroy(sl.rel);
        }
        c.rings.erase(r);
    }
}

}  // namespace nttmi

extern "C" {

ntt_status ntt_forward(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* x, void* X,
                       uint32_t batch, uint32_t flags, void* stream) {
    return ntt_any(false, m, log2n, root, elem_bits, x, X, batch, flags, stream);
}

ntt_status ntt_inverse(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* X, void* x,
                       uint32_t batch, uint32_t flags, void* stream) {
    return ntt_any(true, m, log2n, root, elem_bits, X, x, batch, flags, stream);
}

ntt_status conv_circular(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* f,
                         const void* g, void* h, uint32_t flags, void* stream) {
    int lnu = 0;
    ntt_status st = validate(m, log2n, root, elem_bits, &lnu, flags);
    if (st != NTT_OK) return st;
    if (!f || !g || !h) return NTT_E_ARG;
    const size_t bytes = ((size_t)1 << log2n) * (elem_bits / 8);
    if (overlap(f, bytes, h, bytes) == 2 || overlap(g, bytes, h, bytes) == 2) return NTT_E_ARG;
    if (flags & NTT_FLAG_CHECK_RANGE) {
        st = check_range(elem_bits, f, 1ull << log2n, m, stream);
        if (st == NTT_OK) st = check_range(elem_bits, g, 1ull << log2n, m, stream);
        if (st != NTT_OK) return st;
    }
    const Plan* p = nullptr;
    st = get_plan(m, log2n, root, lnu, &p);
    if (st != NTT_OK) return st;
    return conv_one(p, elem_bits, log2n, f, g, h, stream);
}

ntt_status conv_circular_noalloc(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* f,
                                 const void* g, void* h, uint32_t flags, void* stream) {
    // the checks of validate(), from cached modulus data only
    if (elem_bits != 32 && elem_bits != 64) return NTT_E_ARG;
    if (flags & NTT_FLAG_CHECK_RANGE) return NTT_E_UNSUPPORTED;   // a read-back needs a workspace
    std::pair<int, int> info;
    if (!modulus_info_cached(m, &info)) return NTT_E_NOPLAN;
    int lnu = 0;
    ntt_status st = check_modulus_info(m, elem_bits, info, &lnu, flags);
    if (st != NTT_OK) return st;
    if ((int)log2n > lnu) return NTT_E_LENGTH;
    if (!root_has_order(root, log2n, m)) return NTT_E_ROOT;
    if (log2n > (uint32_t)MAX_LOG2N) return NTT_E_UNSUPPORTED;
    if (!f || !g || !h) return NTT_E_ARG;
    const size_t bytes = ((size_t)1 << log2n) * (elem_bits / 8);
    if (overlap(f, bytes, h, bytes) == 2 || overlap(g, bytes, h, bytes) == 2) return NTT_E_ARG;
    // the four-step scratch: 2N words of the word width
    const bool fourstep = (int)log2n > SMALL_MAX_LOG2N;
    if (fourstep && 2 * bytes > NOALLOC_SCRATCH_BYTES) return NTT_E_UNSUPPORTED;
    const Plan* p = find_plan(m, log2n, root);
    if (!p) return NTT_E_NOPLAN;
    hipStream_t s = (hipStream_t)stream;
    if (!fourstep) {
        count(NTT_COUNT_SMALL);
        return hip_status(launch_conv_small((int)elem_bits, log2n, f, g, h, nullptr, 1, p->dev, s));
    }
    void* ws = nullptr;
    const hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_status(e);
    count(NTT_COUNT_FOURSTEP);
    return hip_status(launch_conv_fourstep((int)elem_bits, log2n, f, g, h, 1, 0, ws, p->dev, s, nullptr,
                                           (uint32_t)cu_count()));
}

ntt_status conv_deconvolve(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits, const void* f,
                           const void* h, void* g, uint32_t batch, uint32_t flags, void* stream) {
    int lnu = 0;
    ntt_status st = validate(m, log2n, root, elem_bits, &lnu, flags);
    if (st != NTT_OK) return st;
    if (batch == 0) return NTT_OK;
    if (!f || !h || !g) return NTT_E_ARG;
    const size_t wb = elem_bits / 8;
    const size_t bytes = ((size_t)batch << log2n) * wb;
    if (overlap(f, bytes, g, bytes) == 2 || overlap(h, bytes, g, bytes) == 2) return NTT_E_ARG;
    // the singular flag is read back with a synchronisation, which a stream
    // being captured cannot do: refuse before anything is enqueued
    bool capturing = false;
    st = stream_capturing(stream, &capturing);
    if (st != NTT_OK) return st;
    if (capturing) return NTT_E_UNSUPPORTED;
    if (flags & NTT_FLAG_CHECK_RANGE) {
        st = check_range(elem_bits, f, (uint64_t)batch << log2n, m, stream);
        if (st == NTT_OK) st = check_range(elem_bits, h, (uint64_t)batch << log2n, m, stream);
        if (st != NTT_OK) return st;
    }
    const Plan* p = nullptr;
    st = get_plan(m, log2n, root, lnu, &p);
    if (st != NTT_OK) return st;
    void* flag = nullptr;
    st = get_buf(caches().flag, stream, sizeof(uint32_t), &flag);
    if (st != NTT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s);
    if (e != hipSuccess) return hip_status(e);
    const char* F = (const char*)f;
    const char* Hh = (const char*)h;
    char* Gg = (char*)g;
    if ((int)log2n <= SMALL_MAX_LOG2N) {
        count(NTT_COUNT_SMALL);
        e = launch_conv_small((int)elem_bits, log2n, F, Hh, Gg, nullptr, batch, p->dev, s, SMALL_TILE_256,
                              (uint32_t*)flag);
    } else {
        // the persistent fused kernel with the quotient as its pointwise step:
        // resident workgroups, each with 2N scratch words, within 1 GiB
        const uint64_t per_wg = ((uint64_t)2 * wb) << log2n;
        uint64_t grid = (uint64_t)std::max(1, cu_count()) * std::max(1, fused_blocks_per_cu((int)elem_bits, log2n, 1));
        grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, (1ull << 30) / per_wg));
        grid = std::min<uint64_t>(grid, batch);
        void* ws = nullptr;
        st = get_buf(caches().work, stream, (size_t)(grid * per_wg), &ws);
        if (st != NTT_OK) return st;
        uint32_t* q = nullptr;
        st = get_queue(stream, &q);
        if (st != NTT_OK) return st;
        count(NTT_COUNT_FUSED);
        e = launch_conv_fused((int)elem_bits, (int)log2n, F, Hh, Gg, nullptr, batch, ws, q, (uint32_t)grid, p->dev, s,
                              (uint32_t*)flag);
    }
    uint32_t hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e);
    return hflag ? NTT_E_SINGULAR : NTT_OK;
}

ntt_status conv_crt(uint32_t log2n, const void* f, const void* g, void* h, uint32_t batch, uint32_t flags,
                    void* stream) {
    (void)flags;
    // the Rader prime 13 2^20 + 1 (root 2^(nu/N)) and the Euler-form prime
    // 7 2^20 + 1 (root z^((m2-1)/N), z = 3 the smallest non-residue)
    const uint64_t m1 = 13631489, m2 = 7340033;
    if (log2n > 19) return NTT_E_LENGTH;
    if (batch == 0) return NTT_OK;
    if (!f || !g || !h) return NTT_E_ARG;
    const uint64_t N = 1ull << log2n;
    const size_t in_bytes = (size_t)batch * N * 4, out_bytes = (size_t)batch * N * 8;
    if (overlap(f, in_bytes, h, out_bytes) || overlap(g, in_bytes, h, out_bytes)) return NTT_E_ARG;
    int l1 = 0, l2 = 0;
    ntt_status st = check_modulus(m1, 32, &l1);
    if (st == NTT_OK) st = check_modulus(m2, 32, &l2, NTT_FLAG_EULER);
    if (st != NTT_OK) return st;
    uint64_t r1 = 0, r2 = 0;
    st = ntt_default_root(m1, log2n, &r1);
    if (st == NTT_OK) st = ntt_euler_root(m2, log2n, &r2);
    if (st != NTT_OK) return st;
    const Plan *p1 = nullptr, *p2 = nullptr;
    st = get_plan(m1, log2n, r1, l1, &p1);
    if (st == NTT_OK) st = get_plan(m2, log2n, r2, l2, &p2);
    if (st != NTT_OK) return st;
    // residues mod m1, then the convolution mod m2 whose final store combines
    // both (the fused kernel's CRT store above 2^12; a combine kernel below)
    void* tmp = nullptr;
    st = get_buf(caches().tune, stream, 2 * in_bytes, &tmp);
    if (st != NTT_OK) return st;
    uint32_t* a1 = (uint32_t*)tmp;
    uint32_t* a2 = a1 + (size_t)batch * N;
    std::vector<uint64_t> off(batch);
    for (uint32_t i = 0; i < batch; ++i) off[i] = (uint64_t)i * N;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t c = (uint32_t)powmod64(m1 % m2, m2 - 2, m2);   // m1^-1 mod m2
    st = launch_class(log2n, off, p1, 32, (const char*)f, (const char*)g, (char*)a1, s, stream);
    if (st != NTT_OK) return st;
    if ((int)log2n > SMALL_MAX_LOG2N) {
        const uint64_t per_wg = (uint64_t)2 * 4 << log2n;
        uint64_t grid = (uint64_t)std::max(1, cu_count()) * std::max(1, fused_blocks_per_cu(32, (int)log2n));
        grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, (1ull << 30) / per_wg));
        grid = std::min<uint64_t>(grid, batch);
        void* ws = nullptr;
        st = get_buf(caches().work, stream, (size_t)(grid * per_wg), &ws);
        if (st != NTT_OK) return st;
        uint32_t* q = nullptr;
        st = get_queue(stream, &q);
        if (st != NTT_OK) return st;
        const CrtStore cs{a1, (uint64_t*)h, (uint32_t)m1, c};
        count(NTT_COUNT_FUSED);
        return hip_status(launch_conv_fused(32, (int)log2n, f, g, nullptr, nullptr, batch, ws, q, (uint32_t)grid,
                                            p2->dev, s, nullptr, &cs));
    }
    st = launch_class(log2n, off, p2, 32, (const char*)f, (const char*)g, (char*)a2, s, stream);
    if (st != NTT_OK) return st;
    return hip_status(launch_crt_combine(a1, a2, (uint64_t*)h, (uint64_t)batch * N, (uint32_t)m1, (uint32_t)m2, c, s));
}

ntt_status conv2d_circular(uint64_t m, uint32_t log2r, uint32_t log2c, uint64_t root_r, uint64_t root_c,
                           uint32_t elem_bits, const void* f, const void* g, void* h, uint32_t flags,
                           void* stream) {
    int lnu = 0;
    ntt_status st = validate(m, log2r, root_r, elem_bits, &lnu, flags);
    if (st == NTT_OK) st = validate(m, log2c, root_c, elem_bits, &lnu, flags);
    if (st != NTT_OK) return st;
    if (log2r + log2c > 31) return NTT_E_UNSUPPORTED;
    if (!f || !g || !h) return NTT_E_ARG;
    const uint32_t R = 1u << log2r, C = 1u << log2c;
    const size_t wb = elem_bits / 8;
    const uint64_t n = (uint64_t)R * C;
    const size_t bytes = (size_t)n * wb;
    if (overlap(f, bytes, h, bytes) == 2 || overlap(g, bytes, h, bytes) == 2) return NTT_E_ARG;
    if (flags & NTT_FLAG_CHECK_RANGE) {
        st = check_range(elem_bits, f, n, m, stream);
        if (st == NTT_OK) st = check_range(elem_bits, g, n, m, stream);
        if (st != NTT_OK) return st;
    }
    const Plan *pr = nullptr, *pc = nullptr;
    st = get_plan(m, log2r, root_r, lnu, &pr);
    if (st == NTT_OK) st = get_plan(m, log2c, root_c, lnu, &pc);
    if (st != NTT_OK) return st;
    void* ws = nullptr;
    st = get_buf(caches().tune, stream, 2 * bytes, &ws);
    if (st != NTT_OK) return st;
    char* A = (char*)ws;
    char* B = A + bytes;
    char* H = (char*)h;
    hipStream_t s = (hipStream_t)stream;
    const int w = (int)elem_bits;
    // forward: rows of f (length C), transpose, rows again (length R); the same
    // for g (h serves as its buffer once f and g have been read); product
    // (formed on load by the next pass for R <= 2^12); inverse along R (with
    // R^-1), transpose back, inverse along C (with C^-1)
    st = ntt_rows(pc, elem_bits, log2c, false, f, A, R, stream);
    if (st == NTT_OK) st = hip_status(launch_transpose(w, A, B, R, C, s));
    if (st == NTT_OK) st = ntt_rows(pr, elem_bits, log2r, false, B, B, C, stream);
    if (st == NTT_OK) st = ntt_rows(pc, elem_bits, log2c, false, g, A, R, stream);
    if (st == NTT_OK) st = hip_status(launch_transpose(w, A, H, R, C, s));
    if (st == NTT_OK) st = ntt_rows(pr, elem_bits, log2r, false, H, H, C, stream);
    if ((int)log2r <= SMALL_MAX_LOG2N) {
        // the product formed on load by the first inverse pass
        if (st == NTT_OK) st = hip_status(launch_ntt_small(w, (int)log2r, true, B, B, C, pr->dev, s, H));
    } else {
        if (st == NTT_OK) st = hip_status(launch_pointwise_mul(w, B, H, B, n, pr->dev.M, s));
        if (st == NTT_OK) st = ntt_rows(pr, elem_bits, log2r, true, B, B, C, stream);
    }
    if (st == NTT_OK) st = hip_status(launch_transpose(w, B, A, C, R, s));
    if (st == NTT_OK) st = ntt_rows(pc, elem_bits, log2c, true, A, H, R, stream);
    return st;
}

ntt_status conv_batched(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                        const ntt_batch_desc* d, const void* f, const void* g, void* h, uint32_t flags,
                        void* stream) {
    int lnu = 0;
    ntt_status st = check_modulus(m, elem_bits, &lnu, flags);
    if (st != NTT_OK) return st;
    if (!d) return NTT_E_ARG;
    if ((int)root_log2order > lnu) return NTT_E_LENGTH;
    if (!root_has_order(root, root_log2order, m)) return NTT_E_ROOT;
    if (d->count == 0) return NTT_OK;
    if (!d->log2n || !d->offset || !f || !g || !h) return NTT_E_ARG;
    const uint32_t cnt = d->count;
    // items: lengths within the root's order, no two items overlapping
    uint64_t total = 0;
    bool ascending = true;   // items listed in address order: overlap is checked in one pass
    bool packed = true;      // one length, items back to back in order
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t n = d->log2n[i];
        if (n > root_log2order) return NTT_E_LENGTH;
        if (n > (uint32_t)MAX_LOG2N) return NTT_E_UNSUPPORTED;
        const uint64_t len = 1ull << n;
        if (d->offset[i] > (UINT64_MAX >> 3) - len) return NTT_E_ARG;
        if (i > 0) {
            const uint64_t prev_end = d->offset[i - 1] + (1ull << d->log2n[i - 1]);
            if (d->offset[i] < prev_end) ascending = false;
            packed = packed && n == d->log2n[0] && d->offset[i] == prev_end;
        }
        total = std::max(total, d->offset[i] + len);
    }
    if (!ascending) {
        std::vector<std::pair<uint64_t, uint64_t>> ext(cnt);
        for (uint32_t i = 0; i < cnt; ++i) ext[i] = std::make_pair(d->offset[i], d->offset[i] + (1ull << d->log2n[i]));
        std::sort(ext.begin(), ext.end());
        for (uint32_t i = 1; i < cnt; ++i)
            if (ext[i].first < ext[i - 1].second) return NTT_E_ARG;
    }
    const size_t bytes = (size_t)total * (elem_bits / 8);
    if (overlap(f, bytes, h, bytes) == 2 || overlap(g, bytes, h, bytes) == 2) return NTT_E_ARG;
    if (flags & NTT_FLAG_CHECK_RANGE) {
        // checks the whole extent, gaps between items included
        st = check_range(elem_bits, f, total, m, stream);
        if (st == NTT_OK) st = check_range(elem_bits, g, total, m, stream);
        if (st != NTT_OK) return st;
    }
    const size_t wb = elem_bits / 8;   // bytes per word
    const char* F = (const char*)f;
    const char* G = (const char*)g;
    char* H = (char*)h;
    hipStream_t s = (hipStream_t)stream;

    // one length, items back to back: launched from the first offset and the
    // count, with no per-length offset lists
    if (packed && !(flags & (NTT_FLAG_PER_ITEM | NTT_FLAG_AUTOTUNE))) {
        const uint32_t n = d->log2n[0];
        const Plan* p = nullptr;
        st = get_plan(m, n, powmod64(root % m, 1ull << (root_log2order - n), m), lnu, &p);
        if (st != NTT_OK) return st;
        BatchForm form;
        uint8_t cf = CF_DEFAULT;
        bool multi = false;   // a tuned form may run the one length in the multi-length kernel
        if (lookup_form(shape_key_uniform(m, elem_bits, n, cnt), &form)) {
            auto it = form.cls.find(n);
            if (it != form.cls.end()) cf = it->second;
            multi = form.multi && !(flags & NTT_FLAG_PER_CLASS) && n <= (uint32_t)multi_max_log2n((int)elem_bits);
        }
        if (!multi) return launch_items(n, cnt, d->offset[0], nullptr, p, elem_bits, F, G, H, s, stream, cf);
    }

    // length classes
    std::map<uint32_t, std::vector<uint64_t>> cls;
    {
        // count per length first, then fill: one allocation per length
        uint32_t per[MAX_LOG2N + 1] = {0};
        for (uint32_t i = 0; i < cnt; ++i) ++per[d->log2n[i]];
        std::vector<uint64_t>* slot[MAX_LOG2N + 1] = {nullptr};
        for (int n = 0; n <= MAX_LOG2N; ++n)
            if (per[n]) {
                slot[n] = &cls[(uint32_t)n];
                slot[n]->reserve(per[n]);
            }
        for (uint32_t i = 0; i < cnt; ++i) slot[d->log2n[i]]->push_back(d->offset[i]);
    }
    std::map<uint32_t, const Plan*> plans;
    for (auto& kv : cls) {
        const uint32_t n = kv.first;
        const uint64_t item_root = powmod64(root % m, 1ull << (root_log2order - n), m);
        const Plan* p = nullptr;
        st = get_plan(m, n, item_root, lnu, &p);
        if (st != NTT_OK) return st;
        plans[n] = p;
    }
    if (flags & NTT_FLAG_PER_ITEM) {
        for (auto& kv : cls)
            for (uint64_t o : kv.second) {
                st = conv_one(plans[kv.first], elem_bits, kv.first, F + o * wb, G + o * wb, H + o * wb, stream);
                if (st != NTT_OK) return st;
            }
        return NTT_OK;
    }
    // Default form: one persistent launch for every length it covers, unless
    // the batch has a single length (whose own kernel may run two workgroups
    // per CU).  A tuned form for this batch shape replaces the default;
    // NTT_FLAG_AUTOTUNE tunes one now.  NTT_FLAG_PER_CLASS forces one launch
    // per length.
    const uint32_t nmax = (uint32_t)multi_max_log2n((int)elem_bits);
    size_t multi_classes = 0;
    uint64_t multi_tasks = 0;
    bool long_contiguous = true;   // every length above the LDS kernels is one back-to-back run
    for (auto& kv : cls) {
        if (kv.first > nmax) continue;
        multi_classes += 1;
        const uint64_t tile = (int)kv.first <= SMALL_MAX_LOG2N ? (uint64_t)multi_tile((int)kv.first) : 1;
        multi_tasks += (kv.second.size() + tile - 1) / tile;
        if ((int)kv.first > SMALL_MAX_LOG2N) {
            const std::vector<uint64_t>& o = kv.second;
            for (size_t i = 1; i < o.size() && long_contiguous; ++i)
                long_contiguous = o[i] == o[0] + ((uint64_t)i << kv.first);
        }
    }
    BatchForm form;
    // The single launch runs one task per workgroup; with fewer tasks than two
    // thirds of its resident workgroups it would leave CUs idle.  Then, when
    // every long length is one back-to-back run, each length's own launch
    // (the four-step form for a few long items) spreads over the chip instead;
    // scattered items (the four-step form needs a uniform stride) keep the
    // single launch.
    const uint64_t resident = (uint64_t)std::max(1, cu_count()) * std::max(1, multi_blocks_per_cu((int)elem_bits));
    form.multi = multi_classes >= 2 && (3 * multi_tasks >= 2 * resident || !long_contiguous);
    const std::vector<uint64_t> key = shape_key(m, elem_bits, cls);
    if (!lookup_form(key, &form) && (flags & NTT_FLAG_AUTOTUNE)) {
        st = autotune(cls, plans, nmax, elem_bits, F, G, H, total, s, stream, &form);
        if (st != NTT_OK) return st;
        store_form(key, form);
    }
    if (flags & NTT_FLAG_PER_CLASS) form.multi = false;
    return run_batch(form, cls, plans, nmax, elem_bits, F, G, H, s, stream, (flags & NTT_FLAG_TRANSIENT) != 0);
}

ntt_status ntt_default_root(uint64_t m, uint32_t log2n, uint64_t* root) {
    if (!root) return NTT_E_ARG;
    const int lnu = modulus_log2nu(m);
    if (lnu < 0) return NTT_E_MODULUS;
    if ((int)log2n > lnu) return NTT_E_LENGTH;
    // 2^(nu/N): the harmonic of exact order N
    *root = powmod64(2, (1ull << lnu) >> log2n, m);
    return NTT_OK;
}

ntt_status ntt_max_log2n(uint64_t m, uint32_t* log2n) {
    if (!log2n) return NTT_E_ARG;
    const int v2 = modulus_info(m).second;
    if (v2 < 0) return NTT_E_MODULUS;
    *log2n = (uint32_t)v2;
    return NTT_OK;
}

ntt_status ntt_euler_root(uint64_t m, uint32_t log2n, uint64_t* root) {
    if (!root) return NTT_E_ARG;
    const int v2 = modulus_info(m).second;
    if (v2 < 0) return NTT_E_MODULUS;
    if ((int)log2n > v2) return NTT_E_LENGTH;
    // the smallest quadratic non-residue z (z^((m-1)/2) = -1); z^((m-1)/N) then
    // has exact order N, since its N/2-th power is z^((m-1)/2)
    uint64_t z = 2;
    while (powmod64(z, (m - 1) / 2, m) != m - 1) ++z;
    *root = powmod64(z, (m - 1) >> log2n, m);
    return NTT_OK;
}

ntt_status ntt_modulus_order(uint64_t m, uint32_t* log2_nu) {
    if (!log2_nu) return NTT_E_ARG;
    const int lnu = modulus_log2nu(m);
    if (lnu < 0) return NTT_E_MODULUS;
    *log2_nu = (uint32_t)lnu;
    return NTT_OK;
}

ntt_status ntt_copy_batch(void* const* dst, const void* const* src, const uint64_t* bytes, uint32_t count,
                          void* stream) {
    if (count == 0) return NTT_OK;
    if (!dst || !src || !bytes) return NTT_E_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (bytes[i] && (!dst[i] || !src[i])) return NTT_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t i = 0; i < count; ++i) {
        if (!bytes[i]) continue;
        hipError_t e = hipMemcpyAsync(dst[i], src[i], (size_t)bytes[i], hipMemcpyDefault, s);
        if (e != hipSuccess) return hip_status(e);
    }
    return NTT_OK;
}

const char* ntt_status_string(ntt_status s) {
    switch (s) {
        case NTT_OK: return "ok";
        case NTT_E_ARG: return "invalid argument (null pointer, element width, descriptor or overlap)";
        case NTT_E_MODULUS: return "invalid modulus (not prime, order of 2 not a power of two, or too wide)";
        case NTT_E_LENGTH: return "length does not divide the order of 2 modulo m";
        case NTT_E_ROOT: return "root is not of exact order N modulo m";
        case NTT_E_RANGE: return "an operand is not below m";
        case NTT_E_NOMEM: return "out of memory";
        case NTT_E_DEVICE: return "HIP runtime or launch failure";
        case NTT_E_UNSUPPORTED: return "valid request not supported by the library";
        case NTT_E_SINGULAR: return "a spectral coefficient of the divisor is zero (no unique quotient)";
        case NTT_E_TIMEOUT: return "the time limit passed before the request finished";
        case NTT_E_NOPLAN: return "no plan for (m, N, root) on this device yet (build it with an earlier call)";
    }
    return "unknown status";
}

void ntt_release_stream(void* stream) { nttmi::release_stream_caches(stream); }

void ntt_launch_counts(uint64_t* counts, uint32_t n) {
    if (!counts) return;
    for (uint32_t k = 0; k < n && k < (uint32_t)NTT_COUNT_SLOTS; ++k) counts[k] = g_counts[k].load(std::memory_order_relaxed);
}

void ntt_release_caches(void) {
    Caches& c = caches();
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : c.plans) {
        if (kv.second.dP) (void)hipFree(kv.second.dP);
        if (kv.second.dTT) (void)hipFree(kv.second.dTT);
        if (kv.second.dTT32) (void)hipFree(kv.second.dTT32);
    }
    c.plans.clear();
    for (auto& kv : c.work) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.work.clear();
    for (auto& kv : c.flag) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.flag.clear();
    for (auto& kv : c.queue) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.queue.clear();
    for (auto& kv : c.tune) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.tune.clear();
    c.forms.clear();
    for (auto& kv : c.offsets) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.offsets.clear();
    for (auto& kv : c.rings)
        for (RingSlot& sl : kv.second.slot) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.rel) (void)hipEventDestroy(sl.rel);
        }
    c.rings.clear();
    for (void* p : c.retired) (void)hipFree(p);
    c.retired.clear();
    for (void* p : c.retired_host) (void)hipHostFree(p);
    c.retired_host.clear();
}

}  // extern "C"
