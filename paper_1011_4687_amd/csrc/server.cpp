// One GPU shared by several host processes (the paper's outlook: Sec. I and
// Sec. V suggest sharing the GPU among the MPI processes of a node).
//
// A server process owns the environments and the GPU.  Clients (other
// processes, e.g. the MPI ranks of a node, or threads) attach to a named
// POSIX shared-memory segment, claim a slot, write a request (environment
// index, points) into it and flag it ready.  The server's worker thread
// gathers every ready slot, copies the points to the device, evaluates all
// requests in one persistent batched launch, copies the potentials back into
// the slots and flags them done.  Clients never call HIP: they only touch
// shared memory, so any number of them can run without a GPU context.
//
// Slot state machine (one 32-bit atomic per slot, acquire/release):
//   IDLE --client writes request--> READY --server evaluates--> DONE/ERROR
//   DONE/ERROR --client reads result--> IDLE
#include <fcntl.h>
#include <signal.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

#include <hip/hip_runtime.h>

#include <atomic>
#include <cerrno>
#include <chrono>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "handle.h"

using namespace envpot;

namespace {

constexpr uint32_t kMagic = 0x45505356u;  // "EPSV"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kIdle = 0, kReady = 1, kDone = 2, kError = 3;

struct ShmHeader {
    uint32_t magic;
    uint32_t version;
    int32_t n_slots;
    int32_t n_env;
    int64_t max_points;
    int64_t slot_stride;      // bytes
    int64_t slot_off;         // bytes from the segment start to slot 0
    int64_t total_bytes;
    int32_t server_pid;
    std::atomic<uint32_t> server_alive;
};

struct SlotHeader {
    std::atomic<uint32_t> owner;   // 0: free, else the client's pid
    std::atomic<uint32_t> state;
    int32_t env;
    int32_t status;
    int64_t n;
    uint64_t seq;
    uint8_t pad[32];
};
static_assert(sizeof(SlotHeader) == 64, "slot header is one cache line");
static_assert(std::atomic<uint32_t>::is_always_lock_free, "process-shared atomics must be lock-free");

std::string shm_name(const char* name) { return std::string("/envpot.") + name; }

bool valid_name(const char* name) {
    if (!name || !*name || std::strlen(name) > 200) return false;
    for (const char* p = name; *p; ++p)
        if (*p == '/') return false;
    return true;
}

inline SlotHeader* slot_at(void* base, const ShmHeader* h, int s) {
    return reinterpret_cast<SlotHeader*>(static_cast<char*>(base) + h->slot_off + int64_t(s) * h->slot_stride);
}
inline double* slot_points(SlotHeader* s) { return reinterpret_cast<double*>(s + 1); }
inline double* slot_out(SlotHeader* s, int64_t max_points) { return slot_points(s) + 3 * max_points; }

void sleep_us(int us) {
    timespec ts{0, long(us) * 1000L};
    nanosleep(&ts, nullptr);
}

}  // namespace

struct env_server {
    std::vector<env_potential*> hs;
    int device = -1;
    // the segment's geometry as the server created it: the header in shared
    // memory is writable by clients, so the server never reads it back
    int32_t n_slots = 0;
    int64_t max_points = 0, slot_off = 0, slot_stride = 0;
    std::string name;
    void* base = nullptr;
    ShmHeader* hdr = nullptr;
    int64_t bytes = 0;
    int32_t gather_us = 0;
    double* d_pts = nullptr;
    double* d_out = nullptr;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::atomic<bool> running{false};
    std::atomic<int64_t> rounds{0}, requests{0}, points{0}, busy_ns{0}, errors{0};
    // batched plans by request set ((slot, environment) per request): a set
    // that comes back with the same point counts replays its captured graph
    std::map<std::vector<int64_t>, env_batch*> plans;
};

struct env_client {
    void* base = nullptr;
    ShmHeader* hdr = nullptr;
    int64_t bytes = 0;
    int slot = -1;
    bool broken = false;
};

namespace {

SlotHeader* server_slot(const env_server* S, int s) {
    return reinterpret_cast<SlotHeader*>(static_cast<char*>(S->base) + S->slot_off + int64_t(s) * S->slot_stride);
}

// One round: evaluate every ready slot in one batched launch.  A slot's
// request (environment, point count) is read once, after its READY state
// was observed with acquire, and only those copies are validated and used:
// a client that rewrites its slot meanwhile cannot move the server out of
// bounds.
void serve_round(env_server* S, std::vector<int>& ready) {
    const int64_t maxp = S->max_points;
    const int32_t n_env = int32_t(S->hs.size());
    std::vector<env_potential*> hs;
    std::vector<const double*> pts;
    std::vector<double*> outs;
    std::vector<int64_t> ns;
    std::vector<int> ids;
    std::vector<int32_t> envs;
    for (int s : ready) {
        SlotHeader* sl = server_slot(S, s);
        const int32_t env = __atomic_load_n(&sl->env, __ATOMIC_RELAXED);
        const int64_t n = __atomic_load_n(&sl->n, __ATOMIC_RELAXED);
        if (env < 0 || env >= n_env || n < 0 || n > maxp) {
            sl->status = ENV_E_ARG;
            S->errors.fetch_add(1);
            sl->state.store(kError, std::memory_order_release);
            continue;
        }
        if (n == 0) {
            sl->status = ENV_OK;
            sl->state.store(kDone, std::memory_order_release);
            continue;
        }
        double* dp = S->d_pts + int64_t(s) * 3 * maxp;
        double* dout = S->d_out + int64_t(s) * maxp;
        if (hipMemcpyAsync(dp, slot_points(sl), size_t(n) * 3 * sizeof(double), hipMemcpyHostToDevice,
                           S->stream) != hipSuccess) {
            sl->status = ENV_E_DEVICE;
            S->errors.fetch_add(1);
            sl->state.store(kError, std::memory_order_release);
            continue;
        }
        hs.push_back(S->hs[env]);
        pts.push_back(dp);
        outs.push_back(dout);
        ns.push_back(n);
        ids.push_back(s);
        envs.push_back(env);
    }
    if (ids.empty()) return;
    std::vector<int64_t> key(ids.size());
    for (size_t k = 0; k < ids.size(); ++k) key[k] = (int64_t(ids[k]) << 32) | envs[k];
    auto it = S->plans.find(key);
    env_status st = ENV_OK;
    if (it == S->plans.end()) {
        if (S->plans.size() >= 256) {  // bounded cache
            for (auto& kv : S->plans) env_batch_destroy(kv.second);
            S->plans.clear();
        }
        env_batch* b = nullptr;
        st = env_batch_create(hs.data(), int32_t(hs.size()), &b);
        if (st == ENV_OK) it = S->plans.emplace(key, b).first;
    }
    if (st == ENV_OK) st = env_batch_eval(it->second, pts.data(), ns.data(), outs.data(), S->stream);
    for (size_t k = 0; k < ids.size(); ++k) {
        SlotHeader* sl = server_slot(S, ids[k]);
        if (st == ENV_OK && hipMemcpyAsync(slot_out(sl, maxp), outs[k], size_t(ns[k]) * sizeof(double),
                                           hipMemcpyDeviceToHost, S->stream) != hipSuccess)
            st = ENV_E_DEVICE;
    }
    if (st == ENV_OK && hipStreamSynchronize(S->stream) != hipSuccess) st = ENV_E_DEVICE;
    int64_t npts = 0;
    for (size_t k = 0; k < ids.size(); ++k) {
        SlotHeader* sl = server_slot(S, ids[k]);
        sl->status = st;
        npts += ns[k];
        sl->state.store(st == ENV_OK ? kDone : kError, std::memory_order_release);
    }
    if (st != ENV_OK) S->errors.fetch_add(int64_t(ids.size()));
    S->rounds.fetch_add(1);
    S->requests.fetch_add(int64_t(ids.size()));
    S->points.fetch_add(npts);
}

void serve(env_server* S) {
    (void)hipSetDevice(S->device);
    std::vector<int> ready;
    int idle_spins = 0;
    while (S->running.load(std::memory_order_acquire)) {
        ready.clear();
        for (int s = 0; s < S->n_slots; ++s)
            if (server_slot(S, s)->state.load(std::memory_order_acquire) == kReady) ready.push_back(s);
        if (ready.empty()) {
            // poll quickly right after work, then back off to 50 us
            sleep_us(idle_spins < 100 ? 2 : 50);
            ++idle_spins;
            continue;
        }
        idle_spins = 0;
        if (S->gather_us > 0) {
            // let other clients' requests of this step arrive, then take them all
            sleep_us(S->gather_us);
            ready.clear();
            for (int s = 0; s < S->n_slots; ++s)
                if (server_slot(S, s)->state.load(std::memory_order_acquire) == kReady) ready.push_back(s);
        }
        const auto t0 = std::chrono::steady_clock::now();
        serve_round(S, ready);
        S->busy_ns.fetch_add(
            std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count());
    }
}

void unmap(void* base, int64_t bytes) {
    if (base) munmap(base, size_t(bytes));
}

}  // namespace

extern "C" {

env_status env_server_create(env_potential* const* hs, int32_t n_env, const char* name, int32_t n_slots,
                             int64_t max_points, int32_t gather_us, env_server** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    if (!hs || n_env <= 0 || !valid_name(name) || n_slots <= 0 || n_slots > 4096 || max_points <= 0 ||
        max_points > (int64_t(1) << 26) || gather_us < 0 || gather_us > 1000000)
        return ENV_E_ARG;
    for (int32_t i = 0; i < n_env; ++i) {
        if (!hs[i]) return ENV_E_ARG;
        if (!hs[i]->on_device) return ENV_E_STATE;
        if (hs[i]->device != hs[0]->device || hs[i]->precision != hs[0]->precision) return ENV_E_ARG;
    }
    const std::string nm = shm_name(name);
    const int64_t stride = ((int64_t(sizeof(SlotHeader)) + 4 * max_points * int64_t(sizeof(double))) + 4095) & ~4095LL;
    const int64_t off = 4096;
    const int64_t bytes = off + stride * n_slots;
    int fd = shm_open(nm.c_str(), O_RDWR | O_CREAT | O_EXCL, 0600);
    if (fd < 0 && errno == EEXIST) {
        // a segment of that name exists: take it over only if its server is gone
        int fo = shm_open(nm.c_str(), O_RDWR, 0600);
        bool stale = true;
        if (fo >= 0) {
            struct stat sb;
            if (fstat(fo, &sb) == 0 && sb.st_size >= off) {
                void* m = mmap(nullptr, size_t(off), PROT_READ, MAP_SHARED, fo, 0);
                if (m != MAP_FAILED) {
                    const ShmHeader* oh = static_cast<const ShmHeader*>(m);
                    if (oh->magic == kMagic && oh->server_alive.load() != 0 &&
                        (kill(oh->server_pid, 0) == 0 || errno != ESRCH))
                        stale = false;
                    munmap(m, size_t(off));
                }
            }
            close(fo);
        }
        if (!stale) return ENV_E_STATE;
        shm_unlink(nm.c_str());
        fd = shm_open(nm.c_str(), O_RDWR | O_CREAT | O_EXCL, 0600);
    }
    if (fd < 0) return ENV_E_STATE;
    if (ftruncate(fd, off_t(bytes)) != 0) {
        close(fd);
        shm_unlink(nm.c_str());
        return ENV_E_NOMEM;
    }
    void* base = mmap(nullptr, size_t(bytes), PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
    close(fd);
    if (base == MAP_FAILED) {
        shm_unlink(nm.c_str());
        return ENV_E_NOMEM;
    }
    env_server* S = new (std::nothrow) env_server;
    if (!S) {
        unmap(base, bytes);
        shm_unlink(nm.c_str());
        return ENV_E_NOMEM;
    }
    S->hs.assign(hs, hs + n_env);
    S->device = hs[0]->device;
    S->name = nm;
    S->base = base;
    S->bytes = bytes;
    S->gather_us = gather_us;
    S->n_slots = n_slots;
    S->max_points = max_points;
    S->slot_off = off;
    S->slot_stride = stride;
    ShmHeader* h = new (base) ShmHeader;
    h->magic = kMagic;
    h->version = kVersion;
    h->n_slots = n_slots;
    h->n_env = n_env;
    h->max_points = max_points;
    h->slot_stride = stride;
    h->slot_off = off;
    h->total_bytes = bytes;
    h->server_pid = int32_t(getpid());
    for (int s = 0; s < n_slots; ++s) {
        SlotHeader* sl = new (slot_at(base, h, s)) SlotHeader;
        sl->owner.store(0);
        sl->state.store(kIdle);
        sl->env = 0;
        sl->status = 0;
        sl->n = 0;
        sl->seq = 0;
    }
    S->hdr = h;
    env_status st = ENV_OK;
    {
        DeviceGuard g(S->device);
        if (hipMalloc(reinterpret_cast<void**>(&S->d_pts), size_t(n_slots) * size_t(max_points) * 3 * sizeof(double)) !=
                hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&S->d_out), size_t(n_slots) * size_t(max_points) * sizeof(double)) !=
                hipSuccess)
            st = ENV_E_NOMEM;
        if (st == ENV_OK && hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) st = ENV_E_DEVICE;
    }
    if (st != ENV_OK) {
        DeviceGuard g(S->device);
        (void)hipFree(S->d_pts);
        (void)hipFree(S->d_out);
        unmap(base, bytes);
        shm_unlink(nm.c_str());
        delete S;
        return st;
    }
    h->server_alive.store(1, std::memory_order_release);
    S->running.store(true, std::memory_order_release);
    try {
        S->worker = std::thread(serve, S);
    } catch (...) {
        h->server_alive.store(0);
        DeviceGuard g(S->device);
        (void)hipStreamDestroy(S->stream);
        (void)hipFree(S->d_pts);
        (void)hipFree(S->d_out);
        unmap(base, bytes);
        shm_unlink(nm.c_str());
        delete S;
        return ENV_E_NOMEM;
    }
    *out = S;
    return ENV_OK;
}

env_status env_server_get_stats(const env_server* S, env_server_stats* st) {
    if (!S || !st) return ENV_E_ARG;
    std::memset(st, 0, sizeof(*st));
    st->rounds = S->rounds.load();
    st->requests = S->requests.load();
    st->points = S->points.load();
    st->busy_seconds = double(S->busy_ns.load()) * 1e-9;
    st->errors = S->errors.load();
    int attached = 0;
    for (int s = 0; s < S->n_slots; ++s)
        if (server_slot(S, s)->owner.load() != 0) ++attached;
    st->clients = attached;
    return ENV_OK;
}

void env_server_destroy(env_server* S) {
    if (!S) return;
    S->running.store(false, std::memory_order_release);
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->plans) env_batch_destroy(kv.second);
    S->plans.clear();
    // requests still waiting get an error and clients see the server gone
    for (int s = 0; s < S->n_slots; ++s) {
        SlotHeader* sl = server_slot(S, s);
        if (sl->state.load(std::memory_order_acquire) == kReady) {
            sl->status = ENV_E_STATE;
            sl->state.store(kError, std::memory_order_release);
        }
    }
    S->hdr->server_alive.store(0, std::memory_order_release);
    shm_unlink(S->name.c_str());
    unmap(S->base, S->bytes);
    {
        DeviceGuard g(S->device);
        (void)hipStreamDestroy(S->stream);
        (void)hipFree(S->d_pts);
        (void)hipFree(S->d_out);
    }
    delete S;
}

env_status env_client_attach(const char* name, env_client** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    if (!valid_name(name)) return ENV_E_ARG;
    const std::string nm = shm_name(name);
    int fd = shm_open(nm.c_str(), O_RDWR, 0600);
    if (fd < 0) return ENV_E_STATE;
    struct stat sb;
    if (fstat(fd, &sb) != 0 || sb.st_size < 4096) {
        close(fd);
        return ENV_E_STATE;
    }
    void* base = mmap(nullptr, size_t(sb.st_size), PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
    close(fd);
    if (base == MAP_FAILED) return ENV_E_NOMEM;
    ShmHeader* h = static_cast<ShmHeader*>(base);
    if (h->magic != kMagic || h->version != kVersion || h->total_bytes != int64_t(sb.st_size) ||
        h->server_alive.load(std::memory_order_acquire) == 0) {
        unmap(base, sb.st_size);
        return ENV_E_STATE;
    }
    const uint32_t me = uint32_t(getpid());
    int slot = -1;
    for (int s = 0; s < h->n_slots && slot < 0; ++s) {
        uint32_t expect = 0;
        if (slot_at(base, h, s)->owner.compare_exchange_strong(expect, me)) slot = s;
    }
    if (slot < 0) {
        unmap(base, sb.st_size);
        return ENV_E_STATE;  // every slot is taken
    }
    env_client* c = new (std::nothrow) env_client;
    if (!c) {
        slot_at(base, h, slot)->owner.store(0);
        unmap(base, sb.st_size);
        return ENV_E_NOMEM;
    }
    SlotHeader* sl = slot_at(base, h, slot);
    sl->state.store(kIdle, std::memory_order_release);
    c->base = base;
    c->hdr = h;
    c->bytes = int64_t(sb.st_size);
    c->slot = slot;
    *out = c;
    return ENV_OK;
}

env_status env_client_info(const env_client* c, int32_t* n_env, int64_t* max_points, int32_t* slot) {
    if (!c) return ENV_E_ARG;
    if (n_env) *n_env = c->hdr->n_env;
    if (max_points) *max_points = c->hdr->max_points;
    if (slot) *slot = c->slot;
    return ENV_OK;
}

env_status env_client_eval(env_client* c, int32_t env, const double* points, int64_t n, double* out,
                           int32_t timeout_ms) {
    if (!c || n < 0 || (n > 0 && (!points || !out))) return ENV_E_ARG;
    if (c->broken) return ENV_E_STATE;
    ShmHeader* h = c->hdr;
    if (env < 0 || env >= h->n_env || n > h->max_points) return ENV_E_ARG;
    if (h->server_alive.load(std::memory_order_acquire) == 0) return ENV_E_STATE;
    SlotHeader* sl = slot_at(c->base, h, c->slot);
    if (n > 0) std::memcpy(slot_points(sl), points, size_t(n) * 3 * sizeof(double));
    sl->env = env;
    sl->n = n;
    sl->status = 0;
    sl->seq += 1;
    sl->state.store(kReady, std::memory_order_release);
    const auto t0 = std::chrono::steady_clock::now();
    int spins = 0;
    uint32_t st;
    for (;;) {
        st = sl->state.load(std::memory_order_acquire);
        if (st == kDone || st == kError) break;
        if (h->server_alive.load(std::memory_order_acquire) == 0) {
            c->broken = true;
            return ENV_E_STATE;
        }
        if (timeout_ms > 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms)) {
            // the request may still be served: this slot cannot be reused
            c->broken = true;
            return ENV_E_DEVICE;
        }
        if (++spins > 64) sleep_us(spins < 2000 ? 5 : 50);
    }
    const env_status r = env_status(sl->status);
    if (st == kDone && r == ENV_OK && n > 0) std::memcpy(out, slot_out(sl, h->max_points), size_t(n) * sizeof(double));
    sl->state.store(kIdle, std::memory_order_release);
    return st == kDone ? r : (r != ENV_OK ? r : ENV_E_DEVICE);
}

void env_client_detach(env_client* c) {
    if (!c) return;
    SlotHeader* sl = slot_at(c->base, c->hdr, c->slot);
    // a slot whose request may still be served stays taken
    if (!c->broken) sl->owner.store(0, std::memory_order_release);
    unmap(c->base, c->bytes);
    delete c;
}

}  // extern "C"
