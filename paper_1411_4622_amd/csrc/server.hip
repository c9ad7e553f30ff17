// Serving many independent SA chains (one slice each) on one GPU.
//
// Resident workgroups (one per chain slot) take requests from a ring of
// descriptors in pinned host memory as soon as they finish the previous
// one, so chains of different sizes and arrival times share the GPU without
// waiting for each other (continuous batching).  The host side admits a
// request only when its PILA (section II-B, Eq. 5; built once per geometry
// and cached) and its chain state fit a fixed device-memory budget that the
// server allocates at creation.
//
// Ring protocol (all words in pinned, coherent host memory):
//  * host: write slot (ticket & mask), then publish tail = ticket + 1 with a
//    release store;
//  * GPU: a workgroup reads tail with a system-scope acquire and claims the
//    next ticket by compare-and-swap on a device-memory counter, so tickets
//    start in order and each exactly once; it records claimed, runs the
//    chain, writes the stats and then done = ticket + 1 with a system-scope
//    release (which also makes the chain's image writes visible);
//  * a workgroup that finds no work for idle_us while no chain of its queue
//    runs (a second device counter counts finished chains) closes the queue
//    by setting the claim counter's top bit, unless a ticket was claimed
//    meanwhile; then every workgroup of the queue leaves and the kernel
//    ends.  The host reopens the queue and relaunches the kernel on a later
//    call when tickets wait and the kernel has ended.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sat_chain.hpp"
#include "sat_host.hpp"

namespace pila {

namespace {

struct RingCtl {
    uint64_t tail;  // tickets published by the host
    uint32_t stop;  // host asks every workgroup to exit when idle
    uint32_t pad;
};

struct alignas(256) RingSlot {
    ChainJob job;
    uint64_t claimed;  // ticket + 1 once a workgroup took it (GPU)
    uint64_t done;     // ticket + 1 once its stats are written (GPU)
    uint64_t cancel;   // ticket + 1 when cancelled (host)
    sat_stats stats;   // (GPU)
};

constexpr int kJobWords = (int)(sizeof(ChainJob) / 4);
static_assert(sizeof(ChainJob) % 4 == 0, "descriptor is copied in 32-bit words");
static_assert(sizeof(sat_stats) % 8 == 0, "stats are copied in 64-bit words");

// BODY kPiped: pipelined body of shape (CPW, E), FP32 chains only; kLong:
// the long-row body (FP32, one estimate per wavefront); kGeneral: the
// general body (any row length, M, precision).
enum { kPiped = 0, kGeneral = 1, kLong = 2 };

// PILA builds and the claim counters' clears run on the null stream, so the
// server adds only its three queue streams to the process.  HIP gives each
// stream one of a few hardware queues (GPU_MAX_HW_QUEUES, 4 by default) and
// a queue runs its work in order: anything behind a resident kernel on the
// same hardware queue waits until that kernel ends.
const hipStream_t kBuildStream = nullptr;

// top bit of a queue's claim counter: the queue's kernel is ending
constexpr unsigned long long kClosed = 1ull << 63;

// before a relaunch: reopen the queue (its previous kernel has ended)
__global__ void reopen_kernel(unsigned long long* head)
{
    if (threadIdx.x == 0) *head &= ~kClosed;
}

template <int BODY, int CPW, int E>
__global__ __launch_bounds__(kPipedThreads) void srv_ring_kernel(RingCtl* ctl, RingSlot* slots,
                                                                 uint32_t mask,
                                                                 unsigned long long* head,
                                                                 int64_t idle_polls, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    __shared__ __align__(16) uint32_t desc[kJobWords];
    __shared__ long long got_s;
    __shared__ uint32_t flags_s[1];
    for (;;) {
        if (threadIdx.x == 0) {
            long long got = -1;
            int64_t idle = 0;
            for (;;) {
                if (__hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                // polled without ordering: an acquire invalidates this XCD's
                // caches, which the chains running beside this workgroup use
                const unsigned long long t =
                    __hip_atomic_load(&ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                const unsigned long long h =
                    __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h & kClosed) break;  // the queue was closed: every workgroup leaves
                if (h < t) {
                    if (atomicCAS(head, h, h + 1) == h) {
                        // acquire once per claim: the slot written before the
                        // tail, and the data the request names, are seen by
                        // this workgroup's later loads
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        got = (long long)h;
                        break;
                    }
                    continue;
                }
                // idle, and no chain of this queue runs: close the queue (the
                // claim counter's top bit), so that all its workgroups leave
                // together and the kernel ends; the compare-and-swap fails if
                // a ticket was claimed meanwhile.  Workgroups never leave one
                // by one: the host relaunches only a kernel that has ended,
                // so a few remaining workgroups would serve every later
                // request alone.
                if (++idle > idle_polls &&
                    __hip_atomic_load(head + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == h &&
                    atomicCAS(head, h, h | kClosed) == h)
                    break;
                __builtin_amdgcn_s_sleep(127);
            }
            got_s = got;
        }
        __syncthreads();
        const long long got = got_s;
        if (got < 0) break;  // the same value in every thread
        RingSlot* sl = &slots[(uint64_t)got & mask];
        const uint32_t* src = (const uint32_t*)&sl->job;
        for (int i = threadIdx.x; i < kJobWords; i += blockDim.x)
            desc[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (threadIdx.x == 0) {
            flags_s[0] = __hip_atomic_load(&sl->cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ==
                         (uint64_t)got + 1;
            __hip_atomic_store(&sl->claimed, (uint64_t)got + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
        const ChainJob J = uniform_job(*(const ChainJob*)desc);
        const bool cancelled = __builtin_amdgcn_readfirstlane(flags_s[0]) != 0;
        const int64_t t0 = (int64_t)wall_clock64();
        if (!cancelled) {
            if constexpr (BODY == kPiped)
                run_chain_piped<float, false, CPW, E, true, true>(J, lds, sh, false);
            else if constexpr (BODY == kLong)
                run_chain_long<float, false, E, true>(J, lds, sh, false);
            else if (J.precision == PILA_F32)
                run_chain_simple_dispatch<float>(J, lds, lds_bytes, sh);
            else
                run_chain_simple_dispatch<double>(J, lds, lds_bytes, sh);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            sat_stats st;
            if (cancelled) {
                __builtin_memset(&st, 0, sizeof(st));
                st.status = PILA_ECANCELED;
            } else {
                st = *J.stats;
            }
            st.t_begin = t0;
            st.t_end = (int64_t)wall_clock64();
            const uint64_t* s64 = (const uint64_t*)&st;
            uint64_t* d64 = (uint64_t*)&sl->stats;
            for (int i = 0; i < (int)(sizeof(sat_stats) / 8); ++i)
                __hip_atomic_store(d64 + i, s64[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            // release: stats and every image write of the chain before done
            __hip_atomic_store(&sl->done, (uint64_t)got + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            atomicAdd(head + 1, 1ull);  // chains finished by this queue
        }
        __syncthreads();
    }
}

typedef void (*RingKernel)(RingCtl*, RingSlot*, uint32_t, unsigned long long*, int64_t, int);

struct RingShape {
    int waves, cpw, e;
    RingKernel k;
};

// the pipelined shape of each workgroup width: M <= waves * cpw, rows <= 64 / cpw * e
const RingShape* ring_shape(int waves)
{
    static const RingShape shapes[] = {{8, 1, 8, srv_ring_kernel<kPiped, 1, 8>},
                                       {4, 2, 8, srv_ring_kernel<kPiped, 2, 8>}};
    for (const RingShape& s : shapes)
        if (s.waves == waves) return &s;
    return nullptr;
}

// the general body's queue: workgroups of 8 wavefronts
const RingShape* general_shape()
{
    static const RingShape g = {8, 1, 0, srv_ring_kernel<kGeneral, 1, 1>};
    return &g;
}

// the long-row body's queue: 8 wavefronts, one estimate each, rows of up to 64 kLongE entries
const RingShape* long_shape()
{
    static const RingShape g = {8, 1, kLongE, srv_ring_kernel<kLong, 1, kLongE>};
    return &g;
}

// ---------------------------------------------------------------------------
// device-memory arena: first fit over a free list, 256-byte granules
// ---------------------------------------------------------------------------
class Arena {
public:
    void init(char* base, size_t bytes)
    {
        base_ = base;
        size_ = bytes;
        free_.clear();
        free_[0] = bytes;
        used_ = 0;
    }
    // offset of a block of at least n bytes, or SIZE_MAX
    size_t alloc(size_t n)
    {
        n = align256(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            used_ += n;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t n)
    {
        n = align256(n ? n : 1);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    char* at(size_t off) const { return base_ + off; }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Block {
    size_t off = SIZE_MAX, len = 0;
};

// one cached PILA (both orders, support, trig) and the geometry it is for
struct PilaEntry {
    std::string key;
    std::vector<double> angles;
    std::vector<uint8_t> mask;
    pila_geom geom;
    pila_csr csr;
    std::vector<Block> blocks;
    int32_t* tcol = nullptr;  // slot words of the entries (pipelined FP32 chains), or NULL
    int refs = 0;
    uint64_t last_use = 0;
};

struct Request {
    PilaEntry* pila = nullptr;
    Block ws;
    bool live = false;
    int32_t body = 0;  // PILA_BODY_* of the queue's kernel for this chain
};

uint64_t mix64(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
    return h * 0xBF58476D1CE4E5B9ULL;
}

std::string geom_key(const pila_geom* g)
{
    std::string k;
    const int32_t head[4] = {g->n, g->n_angles, g->n_bins, g->len_dtype};
    k.append((const char*)head, sizeof(head));
    k.append((const char*)g->angles_deg, sizeof(double) * (size_t)g->n_angles);
    const size_t NP = (size_t)g->n * (size_t)g->n;
    if (g->mask) {
        k.push_back('\1');
        k.append((const char*)g->mask, NP);
    } else {
        k.push_back('\0');
    }
    return k;
}

}  // namespace

}  // namespace pila

using namespace pila;

// one ring: its resident kernel, pinned descriptors and device claim counter
struct Queue {
    const RingShape* shape = nullptr;
    int groups = 0;  // resident workgroups of a launch
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool launched = false;
    int64_t launches = 0;
    RingCtl* ctl = nullptr;  // pinned host memory
    RingSlot* slots = nullptr;
    RingCtl* d_ctl = nullptr;  // device views of the pinned blocks
    RingSlot* d_slots = nullptr;
    unsigned long long* d_head = nullptr;
    uint64_t next = 0;          // local tickets issued
    uint64_t claimed_upto = 0;  // local tickets below this were claimed by the GPU
    std::vector<Request> reqs;  // per slot
};

struct srv_s {
    std::mutex mu;
    srv_config cfg{};
    int device = 0;
    char* arena_base = nullptr;
    Arena arena;
    Block head_blk, scratch_blk;
    size_t fixed_bytes = 0;  // claim counters and build scratch
    uint32_t mask = 0;
    int lds_bytes = 0;
    int64_t idle_polls = 0;
    int64_t reaped = 0;
    uint64_t use_clock = 0;
    Queue q[3];  // kPiped, kGeneral, kLong bodies; ticket = local << 2 | queue
    std::list<std::unique_ptr<PilaEntry>> cache;
};

namespace {

int32_t pila_free(srv_t* s, PilaEntry* e)
{
    for (Block& b : e->blocks)
        if (b.off != SIZE_MAX) s->arena.release(b.off, b.len);
    e->blocks.clear();
    return PILA_OK;
}

// evict the least recently used PILA that no admitted request uses, other than keep
bool evict_one(srv_t* s, const PilaEntry* keep)
{
    auto victim = s->cache.end();
    for (auto it = s->cache.begin(); it != s->cache.end(); ++it) {
        if ((*it)->refs > 0 || it->get() == keep) continue;
        if (victim == s->cache.end() || (*it)->last_use < (*victim)->last_use) victim = it;
    }
    if (victim == s->cache.end()) return false;
    pila_free(s, victim->get());
    s->cache.erase(victim);
    return true;
}

// allocate n bytes, evicting unused PILAs (not keep) while needed
bool alloc_evicting(srv_t* s, size_t n, const PilaEntry* keep, Block* out)
{
    for (;;) {
        const size_t off = s->arena.alloc(n);
        if (off != SIZE_MAX) {
            out->off = off;
            out->len = n;
            return true;
        }
        if (!evict_one(s, keep)) return false;
    }
}

PilaEntry* cache_find(srv_t* s, const std::string& key)
{
    for (auto& e : s->cache)
        if (e->key == key) return e.get();
    return nullptr;
}

// the cached PILA of a geometry, built when absent.  EBUSY when it does not
// fit now (PILAs of admitted requests hold the room), ENOMEM when it could
// not fit even in an otherwise empty budget.
int32_t cache_get(srv_t* s, const pila_geom* g, PilaEntry** out)
{
    std::string key = geom_key(g);
    if (PilaEntry* e = cache_find(s, key)) {
        e->last_use = ++s->use_clock;
        *out = e;
        return PILA_OK;
    }
    const int64_t NP = (int64_t)g->n * g->n, G = (int64_t)g->n_angles * g->n_bins;
    if (pila_build_scratch(g) > s->scratch_blk.len)
        return fail(PILA_ENOMEM, "a %d x %d image exceeds the server's build scratch", g->n, g->n);
    auto e = std::make_unique<PilaEntry>();
    e->key = std::move(key);
    e->angles.assign(g->angles_deg, g->angles_deg + g->n_angles);
    if (g->mask) e->mask.assign(g->mask, g->mask + NP);
    e->geom = *g;
    e->geom.angles_deg = e->angles.data();
    e->geom.mask = g->mask ? e->mask.data() : nullptr;
    std::memset(&e->csr, 0, sizeof(e->csr));
    struct Guard {  // frees the blocks of an entry that is not kept
        srv_t* s;
        PilaEntry* e;
        ~Guard()
        {
            if (e) pila_free(s, e);
        }
    } guard{s, e.get()};
    const size_t ls = g->len_dtype == PILA_F32 ? 4 : 8;
    const size_t sizes1[3] = {sizeof(int64_t) * (size_t)(NP + 1), sizeof(int64_t) * (size_t)(G + 1),
                              sizeof(double) * 2 * (size_t)g->n_angles};
    void** dst1[3] = {(void**)&e->csr.row_ptr, (void**)&e->csr.t_row_ptr, (void**)&e->csr.trig};
    size_t need = 0;
    auto take = [&](const size_t* sz, void*** dst, int n) -> int32_t {
        for (int i = 0; i < n; ++i) need += align256(sz[i]);
        if (need > s->arena.size() - s->fixed_bytes)
            return fail(PILA_ENOMEM, "a %d x %d, %d-angle PILA needs %zu bytes, above the budget",
                        g->n, g->n, g->n_angles, need);
        for (int i = 0; i < n; ++i) {
            Block b;
            if (!alloc_evicting(s, sz[i], e.get(), &b))
                return fail(PILA_EBUSY, "no room for a %d x %d, %d-angle PILA now", g->n, g->n,
                            g->n_angles);
            e->blocks.push_back(b);
            *dst[i] = s->arena.at(b.off);
        }
        return PILA_OK;
    };
    PILA_TRY(take(sizes1, dst1, 3));
    void* scratch = s->arena.at(s->scratch_blk.off);
    PILA_TRY(pila_build_with(&e->geom, &e->csr, scratch, kBuildStream));
    const size_t nnz = (size_t)std::max<int64_t>(e->csr.nnz, 1);
    const size_t sizes2[5] = {4 * nnz, ls * nnz, 4 * nnz, ls * nnz,
                              4 * (size_t)std::max(e->csr.n_support, 1)};
    void** dst2[5] = {(void**)&e->csr.col, &e->csr.len, (void**)&e->csr.t_col, &e->csr.t_len,
                      (void**)&e->csr.support};
    PILA_TRY(take(sizes2, dst2, 5));
    PILA_TRY(pila_build_with(&e->geom, &e->csr, scratch, kBuildStream));
    // FP32 rows the pipelined body can hold: the slot words of the entries
    // for the server's LDS layout (the same for every chain on this PILA)
    if (g->len_dtype == PILA_F32 && e->csr.max_row <= 512 && g->n_angles <= kSlotMaxAngles &&
        piped_allowed(&e->geom, &e->csr)) {
        const size_t sizes3[1] = {sizeof(int32_t) * nnz};
        void** dst3[1] = {(void**)&e->tcol};
        PILA_TRY(take(sizes3, dst3, 1));
        sat_params prm{};
        prm.precision = PILA_F32;
        prm.m_cand = 1;
        prm.n_stages = 1;
        ChainJob J = make_job(&e->geom, &e->csr, nullptr, &prm, nullptr, nullptr);
        hybrid_lds(&J, s->lds_bytes);
        PILA_TRY(launch_tcol(J, e->csr.nnz, e->tcol, kBuildStream));
        // the slot words are read by the queue's kernel on another stream
        PILA_HIP(hipStreamSynchronize(kBuildStream));
    }
    e->last_use = ++s->use_clock;
    *out = e.get();
    guard.e = nullptr;
    s->cache.push_back(std::move(e));
    return PILA_OK;
}

bool queue_running(Queue& q)
{
    if (q.launched && hipEventQuery(q.done_ev) == hipSuccess) q.launched = false;
    return q.launched;
}

int32_t progress_queue(srv_t* s, Queue& q)
{
    // claims happen in ticket order
    while (q.claimed_upto < q.next) {
        const RingSlot& sl = q.slots[q.claimed_upto & s->mask];
        if (__atomic_load_n(&sl.claimed, __ATOMIC_ACQUIRE) != q.claimed_upto + 1) break;
        ++q.claimed_upto;
    }
    if (queue_running(q) || q.claimed_upto >= q.next) return PILA_OK;
    // the kernel has exited (or never ran) while tickets wait: start it
    RingCtl* ctl = q.d_ctl;
    RingSlot* slots = q.d_slots;
    uint32_t mask = s->mask;
    unsigned long long* head = q.d_head;
    int64_t idle = s->idle_polls;
    int lds = s->lds_bytes;
    void* args[] = {&ctl, &slots, &mask, &head, &idle, &lds};
    PILA_TRY(set_lds((const void*)q.shape->k, s->lds_bytes));
    reopen_kernel<<<1, 64, 0, q.stream>>>(head);
    PILA_HIP(hipLaunchKernel((const void*)q.shape->k, dim3((unsigned)q.groups),
                             dim3((unsigned)(q.shape->waves * kWave)), args, (size_t)s->lds_bytes,
                             q.stream));
    PILA_HIP(hipEventRecord(q.done_ev, q.stream));
    q.launched = true;
    ++q.launches;
    return PILA_OK;
}

int32_t progress(srv_t* s)
{
    for (Queue& q : s->q) PILA_TRY(progress_queue(s, q));
    return PILA_OK;
}

void release_request(srv_t* s, Request& rq)
{
    if (rq.ws.off != SIZE_MAX) s->arena.release(rq.ws.off, rq.ws.len);
    rq.ws = Block();
    if (rq.pila) --rq.pila->refs;
    rq.pila = nullptr;
    rq.live = false;
}

// queue and slot of a live ticket
int32_t find_ticket(srv_t* s, uint64_t t, Queue** q, uint64_t* local)
{
    if ((t & 3) > 2) return fail(PILA_ENOTFOUND, "ticket %llu is unknown", (unsigned long long)t);
    Queue& qq = s->q[t & 3];
    const uint64_t l = t >> 2;
    if (l >= qq.next || qq.next - l > (uint64_t)s->cfg.ring_size || !qq.reqs[l & s->mask].live)
        return fail(PILA_ENOTFOUND, "ticket %llu is unknown or already reaped", (unsigned long long)t);
    *q = &qq;
    *local = l;
    return PILA_OK;
}

int32_t destroy_impl(srv_t* s)
{
    int32_t rc = PILA_OK;
    for (Queue& q : s->q) {
        if (!q.ctl) continue;
        for (uint64_t l = q.next > (uint64_t)s->cfg.ring_size ? q.next - s->cfg.ring_size : 0; l < q.next; ++l)
            if (q.reqs[l & s->mask].live) __atomic_store_n(&q.slots[l & s->mask].cancel, l + 1, __ATOMIC_RELEASE);
        __atomic_store_n(&q.ctl->stop, 1u, __ATOMIC_RELEASE);
    }
    for (Queue& q : s->q) {
        if (q.stream && hipStreamSynchronize(q.stream) != hipSuccess) rc = PILA_EHIP;
        if (q.done_ev) (void)hipEventDestroy(q.done_ev);
        if (q.stream) (void)hipStreamDestroy(q.stream);
        if (q.ctl) (void)hipHostFree(q.ctl);
        if (q.slots) (void)hipHostFree(q.slots);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
    return rc;
}

int32_t init_queue(srv_t* s, Queue& q, const RingShape* shape, int groups)
{
    q.shape = shape;
    q.groups = groups;
    q.reqs.resize((size_t)s->cfg.ring_size);
    const size_t off = s->arena.alloc(256);
    if (off == SIZE_MAX) return fail(PILA_ENOMEM, "budget too small");
    q.d_head = (unsigned long long*)s->arena.at(off);
    PILA_HIP(hipHostMalloc((void**)&q.ctl, sizeof(RingCtl), hipHostMallocMapped | hipHostMallocCoherent));
    PILA_HIP(hipHostMalloc((void**)&q.slots, sizeof(RingSlot) * (size_t)s->cfg.ring_size,
                           hipHostMallocMapped | hipHostMallocCoherent));
    std::memset((void*)q.ctl, 0, sizeof(RingCtl));
    std::memset((void*)q.slots, 0, sizeof(RingSlot) * (size_t)s->cfg.ring_size);
    PILA_HIP(hipHostGetDevicePointer((void**)&q.d_ctl, q.ctl, 0));
    PILA_HIP(hipHostGetDevicePointer((void**)&q.d_slots, q.slots, 0));
    PILA_HIP(hipStreamCreateWithFlags(&q.stream, hipStreamNonBlocking));
    PILA_HIP(hipEventCreateWithFlags(&q.done_ev, hipEventDisableTiming));
    PILA_HIP(hipMemsetAsync(q.d_head, 0, 256, kBuildStream));
    return PILA_OK;
}

}  // namespace

extern "C" int32_t srv_create(const srv_config* cfg_in, srv_t** out)
{
    clear_error();
    if (!cfg_in || !out) return fail(PILA_EINVAL, "config or out is NULL");
    *out = nullptr;
    srv_config cfg = *cfg_in;
    if (cfg.waves_per_chain == 0) cfg.waves_per_chain = 8;
    if (cfg.ring_size == 0) cfg.ring_size = 1024;
    if (cfg.idle_us == 0) cfg.idle_us = 20000;
    if (!ring_shape(cfg.waves_per_chain)) return fail(PILA_EINVAL, "waves_per_chain must be 4 or 8");
    if (cfg.ring_size < 1 || (cfg.ring_size & (cfg.ring_size - 1)) || cfg.ring_size > (1 << 20))
        return fail(PILA_EINVAL, "ring_size must be a power of two up to 2^20");
    if (cfg.max_slots < 0 || cfg.idle_us < 0 || cfg.general_slots < 0 || cfg.long_slots < 0)
        return fail(PILA_EINVAL, "negative max_slots, idle_us, general_slots or long_slots");
    if (cfg.mem_budget < ((size_t)1 << 20)) return fail(PILA_ENOMEM, "mem_budget below 1 MiB");
    hipDeviceProp_t prop;
    PILA_TRY(device_props(&prop));
    // default: three quarters of the compute units.  A resident workgroup
    // holds a whole CU (all its LDS and registers), and workgroups of other
    // kernels (the caller's copies, PILA builds) that the dispatcher sends
    // to a fully held XCD wait until one of ours leaves; a quarter of each
    // XCD stays free for them.
    if (cfg.max_slots == 0) cfg.max_slots = std::max(3, prop.multiProcessorCount * 3 / 4);
    if (cfg.max_slots < 3) return fail(PILA_EINVAL, "max_slots must be at least 3");
    // one resident workgroup per compute unit: all LDS but the static part
    size_t stat = 0;
    for (const RingShape* sh : {ring_shape(cfg.waves_per_chain), general_shape(), long_shape()}) {
        hipFuncAttributes fa;
        PILA_HIP(hipFuncGetAttributes(&fa, (const void*)sh->k));
        stat = std::max(stat, fa.sharedSizeBytes);
    }

    srv_s* s = new srv_s();
    auto bail = [&](int32_t rc) {
        std::string msg = pila_last_error();
        destroy_impl(s);
        return fail(rc, "%s", msg.c_str());
    };
    s->cfg = cfg;
    s->lds_bytes = (int)((prop.sharedMemPerBlock - stat - 256) & ~(size_t)255);
    // one poll: ~3.4 us of s_sleep plus a host-memory read
    s->idle_polls = std::max<int64_t>(1, (int64_t)cfg.idle_us / 5);
    s->mask = (uint32_t)cfg.ring_size - 1;
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(PILA_EHIP, "no current device"));
    if (hipMalloc(&s->arena_base, cfg.mem_budget) != hipSuccess)
        return bail(fail(PILA_ENOMEM, "cannot allocate the %zu-byte budget", cfg.mem_budget));
    s->arena.init(s->arena_base, cfg.mem_budget);
    // build scratch for images up to 2048 x 2048 (or what an eighth of the budget allows)
    s->scratch_blk.len = align256(std::min<size_t>(256 + (size_t)2048 * 2048, cfg.mem_budget / 8));
    s->scratch_blk.off = s->arena.alloc(s->scratch_blk.len);
    if (s->scratch_blk.off == SIZE_MAX) return bail(fail(PILA_ENOMEM, "budget too small"));
    // general_slots (default a sixteenth) and long_slots (default a quarter)
    // for those bodies, the pipelined body the rest
    const int gen = cfg.general_slots > 0 ? cfg.general_slots : std::max(1, cfg.max_slots / 16);
    const int lng = cfg.long_slots > 0 ? cfg.long_slots : std::max(1, cfg.max_slots / 4);
    if (gen + lng >= cfg.max_slots)
        return bail(fail(PILA_EINVAL, "general_slots + long_slots must be below max_slots"));
    int32_t rc = init_queue(s, s->q[kPiped], ring_shape(cfg.waves_per_chain), cfg.max_slots - gen - lng);
    if (rc == PILA_OK) rc = init_queue(s, s->q[kGeneral], general_shape(), gen);
    if (rc == PILA_OK) rc = init_queue(s, s->q[kLong], long_shape(), lng);
    if (rc != PILA_OK) return bail(rc);
    if (hipStreamSynchronize(kBuildStream) != hipSuccess)
        return bail(fail(PILA_EHIP, "cannot clear the claim counters"));
    s->fixed_bytes = s->arena.used();
    *out = s;
    return PILA_OK;
}

extern "C" int32_t srv_prepare(srv_t* s, const pila_geom* geom)
{
    clear_error();
    if (!s) return fail(PILA_EINVAL, "server is NULL");
    PILA_TRY(check_geom(geom));
    if (geom->len_dtype == PILA_U8) return fail(PILA_EINVAL, "the server keeps FP32 or FP64 lengths");
    std::lock_guard<std::mutex> lk(s->mu);
    PilaEntry* e = nullptr;
    return cache_get(s, geom, &e);
}

extern "C" int32_t srv_submit(srv_t* s, const srv_request* req, uint64_t* ticket)
{
    clear_error();
    if (!s || !req || !ticket) return fail(PILA_EINVAL, "server, request or ticket is NULL");
    if (!req->d_sino || !req->d_image) return fail(PILA_EINVAL, "sinogram or image is NULL");
    PILA_TRY(check_geom(req->geom));
    if (req->geom->len_dtype == PILA_U8) return fail(PILA_EINVAL, "the server keeps FP32 or FP64 lengths");
    std::lock_guard<std::mutex> lk(s->mu);
    PILA_TRY(progress(s));
    PilaEntry* e = nullptr;
    PILA_TRY(cache_get(s, req->geom, &e));
    PILA_TRY(check_params(&e->geom, &e->csr, &req->params));
    // queue: the pipelined body when the chain fits its shape and LDS, the
    // long-row body for longer rows, else the general body
    const RingShape* ps = s->q[kPiped].shape;
    ChainJob probe = make_job(&e->geom, &e->csr, req->d_sino, &req->params, req->d_image, nullptr);
    // redrawn proposals depend on the image value at the step: general body only
    const bool f32 = req->params.precision == PILA_F32 && req->params.proposal == PILA_PROP_CLAMP;
    int qi = kGeneral;
    if (f32 && e->tcol && piped_allowed(&e->geom, &e->csr) && req->params.m_cand <= ps->waves * ps->cpw &&
        e->csr.max_row <= (kWave / ps->cpw) * ps->e && hybrid_lds(&probe, s->lds_bytes) <= s->lds_bytes)
        qi = kPiped;
    else if (f32 && long_allowed(&e->geom, &e->csr, &req->params) &&
             req->params.m_cand <= long_shape()->waves)
        qi = kLong;
    Queue& q = s->q[qi];
    const uint64_t l = q.next;
    Request& rq = q.reqs[l & s->mask];
    if (rq.live) return fail(PILA_EBUSY, "all %d slots of the ring hold unreaped tickets", s->cfg.ring_size);
    const size_t cb = chain_bytes(&e->geom, &req->params);
    size_t pila_bytes = 0;
    for (const Block& b : e->blocks) pila_bytes += align256(b.len);
    if (align256(cb) + pila_bytes > s->arena.size() - s->fixed_bytes)
        return fail(PILA_ENOMEM, "chain state of %zu bytes and its PILA exceed the budget", cb);
    Block ws;
    if (!alloc_evicting(s, cb, e, &ws)) return fail(PILA_EBUSY, "no room for the chain state now");
    ChainJob J = make_job(&e->geom, &e->csr, req->d_sino, &req->params, req->d_image, s->arena.at(ws.off));
    if (qi == kPiped) {
        hybrid_lds(&J, s->lds_bytes);
        J.tcol = e->tcol;
    }
    if (qi == kLong) long_lds(&J, s->lds_bytes);
    RingSlot& sl = q.slots[l & s->mask];
    J.cancel = &q.d_slots[l & s->mask].cancel;
    J.cancel_tag = l + 1;
    // publish: slot words first, then the tail with a release store (x86
    // keeps the store order; the release keeps the compiler's too)
    std::memcpy((void*)&sl.job, &J, sizeof(J));
    __atomic_store_n(&sl.cancel, (uint64_t)0, __ATOMIC_RELAXED);
    __atomic_store_n(&sl.done, (uint64_t)0, __ATOMIC_RELAXED);
    __atomic_store_n(&sl.claimed, (uint64_t)0, __ATOMIC_RELAXED);
    ++e->refs;
    rq.pila = e;
    rq.ws = ws;
    rq.live = true;
    if (qi == kGeneral) {
        const int64_t rb = (int64_t)J.U * J.K * (J.precision == PILA_F32 ? 4 : 8);
        rq.body = PILA_BODY_GENERAL | (rb <= s->lds_bytes ? 0 : PILA_BODY_GLOBAL_R);
    } else {
        rq.body = (qi == kPiped ? PILA_BODY_PIPED : PILA_BODY_LONG) | PILA_BODY_GLOBAL_R;
    }
    q.next = l + 1;
    __atomic_store_n(&q.ctl->tail, l + 1, __ATOMIC_RELEASE);
    *ticket = (l << 2) | (uint64_t)qi;
    return progress(s);
}

extern "C" int32_t srv_poll(srv_t* s, uint64_t ticket, int32_t* done, sat_stats* stats)
{
    clear_error();
    if (!s || !done) return fail(PILA_EINVAL, "server or done is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *done = 0;
    Queue* q = nullptr;
    uint64_t l = 0;
    PILA_TRY(find_ticket(s, ticket, &q, &l));
    PILA_TRY(progress(s));
    RingSlot& sl = q->slots[l & s->mask];
    if (__atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) != l + 1) return PILA_OK;
    if (stats) {
        std::memcpy(stats, (const void*)&sl.stats, sizeof(sat_stats));
        stats->body = q->reqs[l & s->mask].body;
    }
    release_request(s, q->reqs[l & s->mask]);
    ++s->reaped;
    *done = 1;
    return PILA_OK;
}

extern "C" int32_t srv_cancel(srv_t* s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(PILA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    Queue* q = nullptr;
    uint64_t l = 0;
    PILA_TRY(find_ticket(s, ticket, &q, &l));
    __atomic_store_n(&q->slots[l & s->mask].cancel, l + 1, __ATOMIC_RELEASE);
    return progress(s);
}

extern "C" int32_t srv_get_status(srv_t* s, srv_status* st)
{
    clear_error();
    if (!s || !st) return fail(PILA_EINVAL, "server or status is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    PILA_TRY(progress(s));
    st->submitted = (int64_t)(s->q[0].next + s->q[1].next + s->q[2].next);
    st->reaped = s->reaped;
    st->in_flight = st->submitted - s->reaped;
    st->launches = s->q[0].launches + s->q[1].launches + s->q[2].launches;
    st->bytes_used = s->arena.used();
    st->bytes_budget = s->arena.size();
    st->pila_cached = (int32_t)s->cache.size();
    st->kernel_running = (queue_running(s->q[0]) || queue_running(s->q[1]) || queue_running(s->q[2])) ? 1 : 0;
    return PILA_OK;
}

extern "C" int32_t srv_destroy(srv_t* s)
{
    clear_error();
    if (!s) return PILA_OK;
    const int32_t rc = destroy_impl(s);
    return rc == PILA_OK ? PILA_OK : fail(rc, "a stream failed while the server shut down");
}
