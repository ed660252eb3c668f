// Device build of a handle's pair list and records (devbuild_internal.h).
//
// Stages, each over all pairs at once:
//   1. enumerate and screen every primitive pair of the nonzero blocks
//      (one thread per pair: its block by binary search over the block
//      plan's prefix, its primitives by the block's enumeration order);
//   2. order: stable radix sort by (group, L) -- the enumeration order is
//      already group-major, so kept pairs come out as (group, L, index) and
//      dropped ones after them in enumeration order;
//   3. pair data: product centre, exponent, far-field radius, density-fold
//      entry;
//   4. clusters: one-centre pairs stable-sorted by (atom, radius band); each
//      run is a candidate, accepted when it has two members or more and its
//      members cost more than 1.25 times one merged evaluation; accepted
//      clusters stable-sorted by (group, merged L);
//   5. placement: per-(group, L) counts go to the host, which lays out each
//      group as [pairs by L][clusters by merged L][cluster members] and
//      builds the segments; the device then writes every record, the
//      clusters' member tables and the density-fold tables.
// The density terms of the records stay zero: the fold kernels write them.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "devbuild_internal.h"
#include "envpot_internal.h"
#include "update_internal.h"

#pragma clang force_cuda_host_device begin
#include "screen_math.h"
#pragma clang force_cuda_host_device end

namespace envpot {
namespace {

constexpr int kBuildBlock = 256;

struct BuildArgs {
    int64_t U;                  // primitive pairs enumerated
    int64_t nE;                 // enumerated blocks
    const int64_t* enum_first;  // nE + 1
    const int32_t* enum_blk;
    const int32_t* enum_group;
    const int32_t* blk_IJ;      // per block: I, J
    const double* blk_maxabs;
    const int32_t* sh;          // per shell: atom, l, nprim, 0
    const int64_t* sh_poff;     // per shell: first primitive
    const double* exps;
    const double* coefs;
    const double* n0;
    const double* xyz;          // per atom
    double thr;
    int32_t screen;
    int32_t n_groups;
    int32_t fp64;
    int32_t bands;
    double tfar[kLMax + 1];     // the record's threshold per L (FP32C: the float, widened)
    double w[kLMax + 1];        // estimated cost per L
    double edges[kMaxBands];
    double near_share;
};

struct PairSrc {
    int32_t bk, g, I, J, ia, ib;
};

__host__ __device__ inline int rec_words(int L, bool fp64) { return fp64 ? rec64_words(L) : rec32_words(L); }
__host__ __device__ inline int cl_words(int L, bool fp64) { return fp64 ? cl64_words(L) : cl32_words(L); }

__device__ inline int64_t gid() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }

// Block and primitives of enumerated pair u.
__device__ PairSrc decode_pair(const BuildArgs& a, int64_t u) {
    int64_t lo = 0, hi = a.nE;  // enum_first[lo] <= u < enum_first[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.enum_first[mid] <= u) lo = mid;
        else hi = mid;
    }
    PairSrc s;
    s.bk = a.enum_blk[lo];
    s.g = a.enum_group[lo];
    s.I = a.blk_IJ[2 * s.bk];
    s.J = a.blk_IJ[2 * s.bk + 1];
    const int nI = a.sh[4 * s.I + 2], nJ = a.sh[4 * s.J + 2];
    int64_t r = u - a.enum_first[lo];
    if (s.I != s.J) {
        s.ia = int(r / nJ);
        s.ib = int(r % nJ);
    } else {  // ib >= ia: row ia holds nI - ia pairs
        int i = 0;
        while (r >= nI - i) {
            r -= nI - i;
            ++i;
        }
        s.ia = i;
        s.ib = i + int(r);
    }
    return s;
}

__global__ void k_screen(BuildArgs a, uint32_t* key, uint32_t* val, double* dropb) {
    const int64_t u = gid();
    if (u >= a.U) return;
    const PairSrc s = decode_pair(a, u);
    const int64_t pa = a.sh_poff[s.I] + s.ia, pb = a.sh_poff[s.J] + s.ib;
    const double* A = a.xyz + 3 * int64_t(a.sh[4 * s.I]);
    const double* B = a.xyz + 3 * int64_t(a.sh[4 * s.J]);
    const double bound = sm::screen_bound(a.coefs[pa], a.coefs[pb], a.n0[pa], a.n0[pb], a.exps[pa], a.exps[pb],
                                          sm::dist2(A, B));
    const bool drop = a.screen && bound < a.thr;
    const int L = a.sh[4 * s.I + 1] + a.sh[4 * s.J + 1];
    key[u] = drop ? uint32_t(5 * a.n_groups) : uint32_t(5 * s.g + L);
    val[u] = uint32_t(u);
    const double w = (s.I == s.J && s.ia != s.ib) ? 2.0 : 1.0;
    dropb[u] = drop ? w * a.blk_maxabs[s.bk] * bound : 0.0;
}

// First position of every key of a sorted key array (start[] pre-filled
// with -1; keys index start[] directly).
__global__ void k_key_starts(const uint32_t* key, int64_t n, int64_t* start) {
    const int64_t i = gid();
    if (i >= n) return;
    if (i == 0 || key[i] != key[i - 1]) start[key[i]] = i;
}

__global__ void k_pairs(BuildArgs a, const uint32_t* val, int64_t n_pairs, int64_t n_total, double* pc, double* pp,
                        int32_t* pL, int32_t* pg, int32_t* patom, double* pr2, UpdPair* upd) {
    const int64_t k = gid();
    if (k >= n_total) return;
    const PairSrc s = decode_pair(a, int64_t(val[k]));
    UpdPair q;
    q.blk = s.bk;
    q.ia = int16_t(s.ia);
    q.ib = int16_t(s.ib);
    q.group = s.g;
    q.L = 0;
    q.word = -1;
    if (k < n_pairs) {
        const int L = a.sh[4 * s.I + 1] + a.sh[4 * s.J + 1];
        const double al = a.exps[a.sh_poff[s.I] + s.ia], be = a.exps[a.sh_poff[s.J] + s.ib];
        const double p = al + be;
        const int atI = a.sh[4 * s.I], atJ = a.sh[4 * s.J];
        const double* A = a.xyz + 3 * int64_t(atI);
        const double* B = a.xyz + 3 * int64_t(atJ);
        for (int c = 0; c < 3; ++c) pc[3 * k + c] = atI == atJ ? A[c] : sm::prod_centre(al, A[c], be, B[c], p);
        pp[k] = p;
        pL[k] = L;
        pg[k] = s.g;
        patom[k] = atI == atJ ? atI : -1;
        pr2[k] = sm::rec_r2far(a.tfar[L], p, a.fp64 != 0);
        q.L = L;
    }
    upd[k] = q;
}

// Smallest and largest r2far of the one-centre pairs and their number
// (positive doubles order like their bit patterns).
__global__ void k_r2_range(const int32_t* patom, const double* pr2, int64_t n, unsigned long long* mm) {
    unsigned long long lo = ~0ull, hi = 0ull, cnt = 0ull;
    for (int64_t i = gid(); i < n; i += int64_t(gridDim.x) * blockDim.x) {
        if (patom[i] < 0) continue;
        const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(pr2[i]));
        lo = b < lo ? b : lo;
        hi = b > hi ? b : hi;
        ++cnt;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o), c2 = __shfl_xor(cnt, o);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
        cnt += c2;
    }
    if ((threadIdx.x & 63) == 0 && cnt > 0) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
        atomicAdd(&mm[2], cnt);
    }
}

__global__ void k_cluster_keys(BuildArgs a, const int32_t* patom, const double* pr2, int64_t n,
                               unsigned long long* ckey, uint32_t* cval) {
    const int64_t k = gid();
    if (k >= n) return;
    ckey[k] = patom[k] >= 0
                  ? static_cast<unsigned long long>(patom[k]) * 8ull + unsigned(sm::band_of(pr2[k], a.edges, a.bands))
                  : ~0ull;
    cval[k] = uint32_t(k);
}

__global__ void k_heads(const unsigned long long* ck, int64_t n1, int32_t* head) {
    const int64_t i = gid();
    if (i >= n1) return;
    head[i] = (i == 0 || ck[i] != ck[i - 1]) ? 1 : 0;
}

__global__ void k_run_begin(const int32_t* head, const int32_t* runid, int64_t n1, int64_t* rstart, int64_t* nr) {
    const int64_t i = gid();
    if (i >= n1) return;
    if (head[i]) rstart[runid[i]] = i;
    if (i == n1 - 1) {
        const int64_t m = int64_t(runid[i]) + head[i];
        rstart[m] = n1;
        *nr = m;
    }
}

// One thread per candidate run: the decision, and for an accepted cluster
// its sort key, segment cost term, member words and count.
__global__ void k_runs(BuildArgs a, const int64_t* rstart, const uint32_t* cval, int64_t nr, const int32_t* pL,
                       const int32_t* pg, uint32_t* rkey, uint32_t* rval, double* rterm, int64_t* rmw, int32_t* rn,
                       uint8_t* in_cl, unsigned long long* memb_cnt) {
    const int64_t r = gid();
    if (r >= nr) return;
    const int64_t b = rstart[r], e = rstart[r + 1];
    int Lc = 0;
    double cost = 0.0;
    for (int64_t i = b; i < e; ++i) {
        const int L = pL[cval[i]];
        Lc = L > Lc ? L : Lc;
        cost += a.w[L];
    }
    rval[r] = uint32_t(r);
    if (!(e - b >= 2 && cost > 1.25 * a.w[Lc])) {
        rkey[r] = uint32_t(8 * a.n_groups);
        rterm[r] = 0.0;
        rmw[r] = 0;
        rn[r] = 0;
        return;
    }
    const int g = pg[cval[b]];
    rkey[r] = uint32_t(8 * g + Lc);
    int64_t mw = 0;
    int cnt[kLMax + 1] = {0, 0, 0, 0, 0};
    for (int64_t i = b; i < e; ++i) {
        const uint32_t k = cval[i];
        const int L = pL[k];
        mw += rec_words(L, a.fp64 != 0);
        ++cnt[L];
        in_cl[k] = 1;
    }
    for (int L = 0; L <= kLMax; ++L)
        if (cnt[L]) atomicAdd(&memb_cnt[5 * g + L], static_cast<unsigned long long>(cnt[L]));
    // the members are in index order, which is L order within a group: their
    // cost summed in the packer's member order is the same sum
    rterm[r] = sm::cluster_term(a.w[Lc], a.near_share, cost);
    rmw[r] = mw;
    rn[r] = int32_t(e - b);
}

__global__ void k_gather_runs(const uint32_t* cl_run, int64_t nC, const double* rterm, const int64_t* rmw,
                              const int32_t* rn, double* ct, int64_t* cmw, int32_t* cn) {
    const int64_t c = gid();
    if (c >= nC) return;
    const uint32_t r = cl_run[c];
    ct[c] = rterm[r];
    cmw[c] = rmw[r];
    cn[c] = rn[r];
}

__global__ void k_not_in_cluster(const uint8_t* in_cl, int64_t n, int32_t* f) {
    const int64_t k = gid();
    if (k >= n) return;
    f[k] = in_cl[k] ? 0 : 1;
}

__global__ void k_place_pairs(const int32_t* pL, const int32_t* pg, const uint8_t* in_cl, const int32_t* orank,
                              const int64_t* pstart, const int64_t* ooff, int64_t n, int fp64, UpdPair* upd) {
    const int64_t k = gid();
    if (k >= n || in_cl[k]) return;
    const int key = 5 * pg[k] + pL[k];
    const int64_t rank = int64_t(orank[k]) - int64_t(orank[pstart[key]]);
    upd[k].word = ooff[key] + rank * rec_words(pL[k], fp64 != 0);
}

// One thread per accepted cluster: member words and tables, the cluster
// record, its density-fold entry.
__global__ void k_place_clusters(int fp64, const uint32_t* cl_run, const int64_t* rstart, const uint32_t* cval,
                                 const int64_t* cword, const int64_t* mbase, const int64_t* mpos, int64_t nC,
                                 const int32_t* pL, const double* pc, const double* pr2, UpdPair* upd,
                                 int64_t* members, UpdCluster* ucl, uint32_t* rec, int64_t words) {
    const int64_t c = gid();
    if (c >= nC) return;
    const uint32_t r = cl_run[c];
    const int64_t b = rstart[r], e = rstart[r + 1];
    int64_t word = mbase[c], pos = mpos[c];
    int64_t off[kLMax + 1] = {0, 0, 0, 0, 0}, cnt[kLMax + 1] = {0, 0, 0, 0, 0};
    double r2 = 0.0;
    int Lc = 0;
    for (int64_t i = b; i < e; ++i, ++pos) {
        const uint32_t k = cval[i];
        const int L = pL[k];
        if (cnt[L] == 0) off[L] = word;
        ++cnt[L];
        upd[k].word = word;
        members[pos] = int64_t(k);
        word += rec_words(L, fp64 != 0);
        r2 = pr2[k] > r2 ? pr2[k] : r2;
        Lc = L > Lc ? L : Lc;
    }
    const uint32_t k0 = cval[b];
    const int64_t o = cword[c];
    if (o < 0 || o + cl_words(Lc, fp64 != 0) > words) return;  // placed by the host tables; never taken
    uint32_t mask = 0;
    for (int L = 0; L <= kLMax; ++L) mask |= cnt[L] ? (1u << L) : 0u;
    double* d = reinterpret_cast<double*>(rec + o);
    d[0] = pc[3 * int64_t(k0)];
    d[1] = pc[3 * int64_t(k0) + 1];
    d[2] = pc[3 * int64_t(k0) + 2];
    const int mk = fp64 ? kClMask64 : kClMask32, tab = fp64 ? kClTable64 : kClTable32;
    if (fp64) d[3] = r2;
    else reinterpret_cast<float*>(rec + o)[6] = float(r2);
    rec[o + mk] = mask;
    for (int L = 0; L <= kLMax; ++L) {
        rec[o + tab + 2 * L] = uint32_t(off[L]);
        rec[o + tab + 2 * L + 1] = uint32_t(cnt[L]);
    }
    UpdCluster u;
    u.word = o;
    u.begin = mpos[c];
    u.end = mpos[c] + (e - b);
    u.L = Lc;
    u.pad = 0;
    ucl[c] = u;
}

__global__ void k_pair_records(const UpdPair* upd, const double* pc, const double* pp, const double* pr2,
                               const int32_t* pL, int64_t n, int fp64, uint32_t* rec, int64_t words) {
    const int64_t k = gid();
    if (k >= n) return;
    const int64_t o = upd[k].word;
    if (o < 0 || o + rec_words(pL[k], fp64 != 0) > words) return;  // every pair is placed; never taken
    const double p = pp[k];
    double* d = reinterpret_cast<double*>(rec + o);
    d[0] = pc[3 * k];
    d[1] = pc[3 * k + 1];
    d[2] = pc[3 * k + 2];
    if (fp64) {
        d[3] = pr2[k];
        d[4] = p;
        d[5] = sm::rec_c1(p);
    } else {
        float* f = reinterpret_cast<float*>(rec + o + 6);
        f[0] = float(pr2[k]);
        f[1] = float(p);
        f[2] = float(sm::rec_c1(p));
    }
}

__global__ void k_member_sizes(const int64_t* members, const int32_t* pL, int64_t nM, int64_t* sz) {
    const int64_t m = gid();
    if (m >= nM) return;
    sz[m] = kNComp[pL[members[m]]];
}

unsigned grid_of(int64_t n) { return unsigned((n + kBuildBlock - 1) / kBuildBlock); }

// Number of entries of each key from the first positions of the keys in a
// sorted array of n keys (-1: key absent).
std::vector<int64_t> counts_of(const std::vector<int64_t>& start, int64_t n) {
    std::vector<int64_t> c(start.size(), 0);
    int64_t next = n;
    for (int64_t k = int64_t(start.size()) - 1; k >= 0; --k)
        if (start[k] >= 0) {
            c[k] = next - start[k];
            next = start[k];
        }
    return c;
}

int end_bit_above(uint64_t max_key) {  // smallest b with 2^b > max_key
    int b = 1;
    while (b < 64 && (uint64_t(1) << b) <= max_key) ++b;
    return b;
}

// Device allocations of one build; whatever is not released to the caller
// is freed on exit.
struct Arena {
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    template <class T>
    T* alloc(int64_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, size_t(std::max<int64_t>(n, 1)) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        bytes += std::max<int64_t>(n, 1) * int64_t(sizeof(T));
        return static_cast<T*>(p);
    }
    template <class T>
    T* upload(const std::vector<T>& v) {
        T* p = alloc<T>(int64_t(v.size()));
        if (p && !v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return nullptr;
        return p;
    }
    void release(void* p) {  // hand over to the caller
        ptrs.erase(std::remove(ptrs.begin(), ptrs.end(), p), ptrs.end());
    }
    ~Arena() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

// Copy n elements to the host after the stream's work so far.
template <class T>
bool download(std::vector<T>& v, const T* d, int64_t n, hipStream_t st) {
    v.resize(size_t(n));
    if (n == 0) return true;
    return hipMemcpyAsync(v.data(), d, size_t(n) * sizeof(T), hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
}

template <class T>
bool download1(T* v, const T* d, hipStream_t st) {
    return hipMemcpyAsync(v, d, sizeof(T), hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
}

#define DB_CHECK(x)                                  \
    do {                                             \
        if (!(x)) return ENV_E_DEVICE;               \
    } while (0)
#define DB_LAUNCH(n, kern, ...)                                                                  \
    do {                                                                                         \
        if ((n) > 0) {                                                                           \
            hipLaunchKernelGGL(kern, dim3(grid_of(n)), dim3(kBuildBlock), 0, st, __VA_ARGS__);      \
            if (hipGetLastError() != hipSuccess) return ENV_E_DEVICE;                            \
        }                                                                                        \
    } while (0)

}  // namespace

bool device_build_fits(const BlockPlan& plan, const PairList& meta, int n_nuclei) {
    const int64_t U = plan.enum_first.empty() ? 0 : plan.enum_first.back();
    return U < (int64_t(1) << 31) && int64_t(meta.n_groups) * 8 + 1 < (int64_t(1) << 31) &&
           int64_t(n_nuclei) < (int64_t(1) << 58) && int64_t(plan.enum_blk.size()) < (int64_t(1) << 31);
}

void free_device_build(DevBuild& b) {
    (void)hipFree(b.d_rec);
    (void)hipFree(b.d_pairs);
    (void)hipFree(b.d_clusters);
    (void)hipFree(b.d_members);
    (void)hipFree(b.d_moff);
    b.d_rec = nullptr;
    b.d_pairs = nullptr;
    b.d_clusters = nullptr;
    b.d_members = nullptr;
    b.d_moff = nullptr;
}

env_status device_build(const BlockPlan& plan, const PairSources& src, const PairList& meta, bool fp64,
                        const BoysParams& bp, bool merge, DevBuild& out) {
    out = DevBuild();
    Arena ar;
    // the build's own stream (default priority): its work and copies wait
    // for nothing else on the device, and nothing else waits for them
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return ENV_E_DEVICE;
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } stream_guard{st};
    const char* tenv = std::getenv("ENVPOT_TIMING");
    const bool timing = tenv && *tenv && *tenv != '0';
    auto tlast = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {  // waits for the device when timing
        if (!timing) return;
        (void)hipStreamSynchronize(st);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[envpot device build] %-16s %8.3f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - tlast).count());
        tlast = now;
    };
    const int nG = meta.n_groups;
    const int64_t U = plan.enum_first.back();
    const int64_t nE = int64_t(plan.enum_blk.size());
    const int n_shells = int(src.shell_l.size());
    const int n_atoms = int(src.atom_xyz.size() / 3);
    out.n_unscreened = U;
    out.group_pair_begin.assign(size_t(nG) + 1, 0);

    // ---- inputs
    std::vector<int32_t> blk_IJ(2 * src.blk_I.size()), sh(4 * size_t(n_shells), 0);
    for (size_t b = 0; b < src.blk_I.size(); ++b) {
        blk_IJ[2 * b] = src.blk_I[b];
        blk_IJ[2 * b + 1] = src.blk_J[b];
    }
    for (int s = 0; s < n_shells; ++s) {
        sh[4 * s] = src.shell_atom[s];
        sh[4 * s + 1] = src.shell_l[s];
        sh[4 * s + 2] = plan.shell_nprim[s];
    }
    BuildArgs a{};
    a.U = U;
    a.nE = nE;
    a.enum_first = ar.upload(plan.enum_first);
    a.enum_blk = ar.upload(plan.enum_blk);
    a.enum_group = ar.upload(plan.enum_group);
    a.blk_IJ = ar.upload(blk_IJ);
    a.blk_maxabs = ar.upload(plan.blk_maxabs);
    a.sh = ar.upload(sh);
    a.sh_poff = ar.upload(src.poff);
    a.exps = ar.upload(src.exps);
    a.coefs = ar.upload(plan.coefs);
    a.n0 = ar.upload(plan.n0);
    a.xyz = ar.upload(src.atom_xyz);
    if (!a.enum_first || !a.enum_blk || !a.enum_group || !a.blk_IJ || !a.blk_maxabs || !a.sh || !a.sh_poff ||
        !a.exps || !a.coefs || !a.n0 || !a.xyz)
        return ENV_E_NOMEM;
    a.thr = plan.thr;
    a.screen = plan.screen ? 1 : 0;
    a.n_groups = nG;
    a.fp64 = fp64 ? 1 : 0;
    a.bands = radius_bands();
    const double* wc = fp64 ? kCost64 : kCost32;
    for (int L = 0; L <= kLMax; ++L) {
        a.tfar[L] = fp64 ? bp.tfar64[L] : double(bp.tfar32[L]);
        a.w[L] = wc[L];
    }
    a.near_share = kClusterNearShare;

    // ---- 1-2. screen and order
    uint32_t* key = ar.alloc<uint32_t>(U);
    uint32_t* val = ar.alloc<uint32_t>(U);
    uint32_t* key_s = ar.alloc<uint32_t>(U);
    uint32_t* val_s = ar.alloc<uint32_t>(U);
    double* dropb = ar.alloc<double>(U);
    double* d_sb = ar.alloc<double>(1);
    int64_t* pstart = ar.alloc<int64_t>(5 * int64_t(nG) + 1);
    if (!key || !val || !key_s || !val_s || !dropb || !d_sb || !pstart) return ENV_E_NOMEM;
    DB_LAUNCH(U, k_screen, a, key, val, dropb);
    DB_CHECK(hipMemsetAsync(pstart, 0xff, (5 * size_t(nG) + 1) * sizeof(int64_t), st) == hipSuccess);
    if (U > 0) {
        const int eb = end_bit_above(uint64_t(5) * nG);
        size_t tb = 0;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key_s, val, val_s, int(U), 0, eb, st) ==
                 hipSuccess);
        void* tmp = ar.alloc<char>(int64_t(tb));
        if (!tmp) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key_s, val, val_s, int(U), 0, eb, st) ==
                 hipSuccess);
        size_t tr = 0;
        DB_CHECK(hipcub::DeviceReduce::Sum(nullptr, tr, dropb, d_sb, int(U), st) == hipSuccess);
        void* tmp2 = ar.alloc<char>(int64_t(tr));
        if (!tmp2) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceReduce::Sum(tmp2, tr, dropb, d_sb, int(U), st) == hipSuccess);
        DB_CHECK(download1(&out.screened_bound, d_sb, st));
    }
    DB_LAUNCH(U, k_key_starts, key_s, U, pstart);
    lap("upload, screen, sort");
    std::vector<int64_t> hstart;
    DB_CHECK(download(hstart, pstart, 5 * int64_t(nG) + 1, st));
    const std::vector<int64_t> pcount = counts_of(hstart, U);
    const int64_t n_dropped = pcount[5 * size_t(nG)];
    const int64_t n_pairs = U - n_dropped;
    const int64_t n_drop = src.neutralize ? n_dropped : 0;
    out.n_pairs = n_pairs;
    out.n_drop = n_drop;
    for (int g = 0; g < nG; ++g) {
        int64_t s = 0;
        for (int L = 0; L <= kLMax; ++L) {
            s += pcount[5 * g + L];
            out.n_pairs_by_L[L] += pcount[5 * g + L];
        }
        out.group_pair_begin[g + 1] = out.group_pair_begin[g] + s;
    }

    // ---- 3. pair data and the density-fold entries
    double* pc = ar.alloc<double>(3 * n_pairs);
    double* pp = ar.alloc<double>(n_pairs);
    int32_t* pL = ar.alloc<int32_t>(n_pairs);
    int32_t* pg = ar.alloc<int32_t>(n_pairs);
    int32_t* patom = ar.alloc<int32_t>(n_pairs);
    double* pr2 = ar.alloc<double>(n_pairs);
    UpdPair* upd = ar.alloc<UpdPair>(n_pairs + n_drop);
    uint8_t* in_cl = ar.alloc<uint8_t>(n_pairs);
    unsigned long long* memb_cnt = ar.alloc<unsigned long long>(5 * int64_t(std::max(nG, 1)));
    if (!pc || !pp || !pL || !pg || !patom || !pr2 || !upd || !in_cl || !memb_cnt) return ENV_E_NOMEM;
    DB_LAUNCH(n_pairs + n_drop, k_pairs, a, val_s, n_pairs, n_pairs + n_drop, pc, pp, pL, pg, patom, pr2, upd);
    if (n_drop > 0) {
        std::vector<UpdPair> dr;
        DB_CHECK(download(dr, upd + n_pairs, n_drop, st));
        out.drop_group.resize(size_t(n_drop));
        for (int64_t j = 0; j < n_drop; ++j) out.drop_group[j] = dr[j].group;
    }

    lap("pair data");
    // ---- 4. clusters
    DB_CHECK(hipMemsetAsync(in_cl, 0, size_t(std::max<int64_t>(n_pairs, 1)), st) == hipSuccess);
    DB_CHECK(hipMemsetAsync(memb_cnt, 0, 5 * size_t(std::max(nG, 1)) * sizeof(unsigned long long), st) == hipSuccess);
    int64_t n1 = 0, nr = 0, nC = 0;
    uint32_t* cval_s = nullptr;
    int64_t* rstart = nullptr;
    uint32_t* cl_run = nullptr;
    std::vector<int64_t> hcstart;
    std::vector<double> ct;
    std::vector<int64_t> cmw;
    std::vector<int32_t> cn;
    if (merge && n_pairs > 0) {
        unsigned long long* mm = ar.alloc<unsigned long long>(3);
        if (!mm) return ENV_E_NOMEM;
        const unsigned long long init[3] = {~0ull, 0ull, 0ull};
        DB_CHECK(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, st) == hipSuccess);
        hipLaunchKernelGGL(k_r2_range, dim3(std::min<unsigned>(grid_of(n_pairs), 2048u)), dim3(kBuildBlock), 0,
                           st, patom, pr2, n_pairs, mm);
        DB_CHECK(hipGetLastError() == hipSuccess);
        unsigned long long hm[3];
        DB_CHECK(hipMemcpyAsync(hm, mm, sizeof(hm), hipMemcpyDeviceToHost, st) == hipSuccess &&
                 hipStreamSynchronize(st) == hipSuccess);
        n1 = int64_t(hm[2]);
        if (n1 > 0) {
            double vmin, vmax;
            std::memcpy(&vmin, &hm[0], sizeof(double));
            std::memcpy(&vmax, &hm[1], sizeof(double));
            radius_band_edges(vmin, vmax, a.bands, a.edges);
        }
    }
    if (n1 > 0) {
        unsigned long long* ck = ar.alloc<unsigned long long>(n_pairs);
        unsigned long long* ck_s = ar.alloc<unsigned long long>(n_pairs);
        uint32_t* cv = ar.alloc<uint32_t>(n_pairs);
        cval_s = ar.alloc<uint32_t>(n_pairs);
        int32_t* head = ar.alloc<int32_t>(n1);
        int32_t* runid = ar.alloc<int32_t>(n1);
        rstart = ar.alloc<int64_t>(n1 + 1);
        int64_t* d_nr = ar.alloc<int64_t>(1);
        if (!ck || !ck_s || !cv || !cval_s || !head || !runid || !rstart || !d_nr) return ENV_E_NOMEM;
        DB_LAUNCH(n_pairs, k_cluster_keys, a, patom, pr2, n_pairs, ck, cv);
        const int eb = end_bit_above(uint64_t(n_atoms) * 8ull);
        size_t tb = 0;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, ck, ck_s, cv, cval_s, int(n_pairs), 0, eb, st) ==
                 hipSuccess);
        void* tmp = ar.alloc<char>(int64_t(tb));
        if (!tmp) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, ck, ck_s, cv, cval_s, int(n_pairs), 0, eb, st) ==
                 hipSuccess);
        DB_LAUNCH(n1, k_heads, ck_s, n1, head);
        size_t ts = 0;
        DB_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, ts, head, runid, int(n1), st) == hipSuccess);
        void* tmp2 = ar.alloc<char>(int64_t(ts));
        if (!tmp2) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp2, ts, head, runid, int(n1), st) == hipSuccess);
        DB_LAUNCH(n1, k_run_begin, head, runid, n1, rstart, d_nr);
        DB_CHECK(download1(&nr, d_nr, st));

        uint32_t* rkey = ar.alloc<uint32_t>(nr);
        uint32_t* rval = ar.alloc<uint32_t>(nr);
        uint32_t* rkey_s = ar.alloc<uint32_t>(nr);
        cl_run = ar.alloc<uint32_t>(nr);
        double* rterm = ar.alloc<double>(nr);
        int64_t* rmw = ar.alloc<int64_t>(nr);
        int32_t* rn = ar.alloc<int32_t>(nr);
        int64_t* cstart = ar.alloc<int64_t>(8 * int64_t(nG) + 1);
        if (!rkey || !rval || !rkey_s || !cl_run || !rterm || !rmw || !rn || !cstart) return ENV_E_NOMEM;
        DB_LAUNCH(nr, k_runs, a, rstart, cval_s, nr, pL, pg, rkey, rval, rterm, rmw, rn, in_cl, memb_cnt);
        const int eb2 = end_bit_above(uint64_t(8) * nG);
        size_t tb2 = 0;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, rkey, rkey_s, rval, cl_run, int(nr), 0, eb2,
                                                    st) == hipSuccess);
        void* tmp3 = ar.alloc<char>(int64_t(tb2));
        if (!tmp3) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp3, tb2, rkey, rkey_s, rval, cl_run, int(nr), 0, eb2,
                                                    st) == hipSuccess);
        DB_CHECK(hipMemsetAsync(cstart, 0xff, (8 * size_t(nG) + 1) * sizeof(int64_t), st) == hipSuccess);
        DB_LAUNCH(nr, k_key_starts, rkey_s, nr, cstart);
        DB_CHECK(download(hcstart, cstart, 8 * int64_t(nG) + 1, st));
        nC = hcstart[8 * size_t(nG)] >= 0 ? hcstart[8 * size_t(nG)] : nr;
        double* d_ct = ar.alloc<double>(nC);
        int64_t* d_cmw = ar.alloc<int64_t>(nC);
        int32_t* d_cn = ar.alloc<int32_t>(nC);
        if (!d_ct || !d_cmw || !d_cn) return ENV_E_NOMEM;
        DB_LAUNCH(nC, k_gather_runs, cl_run, nC, rterm, rmw, rn, d_ct, d_cmw, d_cn);
        DB_CHECK(download(ct, d_ct, nC, st) && download(cmw, d_cmw, nC, st) && download(cn, d_cn, nC, st));
    }

    lap("clusters");
    // ---- 5. per-group layout on the host
    std::vector<unsigned long long> hmemb;
    DB_CHECK(download(hmemb, memb_cnt, 5 * int64_t(nG), st));
    const std::vector<int64_t> ccount = nC > 0 ? counts_of(hcstart, nr) : std::vector<int64_t>(8 * size_t(nG) + 1, 0);
    std::vector<int64_t> ooff(5 * size_t(nG), 0), cword(size_t(nC), 0), mbase(size_t(nC), 0),
        mpos(size_t(nC) + 1, 0);
    const double* w = a.w;
    int64_t words = 0;
    for (int64_t c = 0; c < nC; ++c) mpos[c + 1] = mpos[c] + cn[c];
    for (int g = 0; g < nG; ++g) {
        const int64_t base = words;
        int64_t oc[kLMax + 1], cc[kLMax + 1], cfirst[kLMax + 1];
        int64_t ow = 0, cw = 0;
        for (int L = 0; L <= kLMax; ++L) {
            oc[L] = pcount[5 * g + L] - int64_t(hmemb[5 * g + L]);
            ooff[5 * g + L] = base + ow;
            ow += oc[L] * rec_words(L, fp64);
        }
        int64_t cbeg = -1, cend = -1;
        for (int L = 0; L <= kLMax; ++L) {
            cc[L] = ccount[8 * size_t(g) + L];
            cfirst[L] = cc[L] > 0 ? hcstart[8 * size_t(g) + L] : -1;
            if (cc[L] > 0) {
                if (cbeg < 0) cbeg = cfirst[L];
                cend = cfirst[L] + cc[L];
            }
        }
        for (int L = 0; L <= kLMax; ++L) {
            for (int64_t j = 0; j < cc[L]; ++j) cword[cfirst[L] + j] = base + ow + cw + j * cl_words(L, fp64);
            cw += cc[L] * cl_words(L, fp64);
        }
        int64_t mw = 0;
        for (int64_t c = cbeg; c >= 0 && c < cend; ++c) {
            mbase[c] = base + ow + cw + mw;
            mw += cmw[c];
        }
        // segments, as the host packer makes them
        const size_t first_seg = out.base.size();
        for (int L = 0; L <= kLMax; ++L) {
            if (oc[L] <= 0) continue;
            Segment sg{};
            sg.L = L;
            sg.n_pairs = int32_t(oc[L]);
            sg.rec_off = ooff[5 * g + L];
            out.base.push_back(sg);
            out.unit_cost.push_back(w[L]);
        }
        for (int L = 0; L <= kLMax; ++L) {
            if (cc[L] <= 0) continue;
            Segment sg{};
            sg.L = L;
            sg.n_pairs = int32_t(cc[L]);
            sg.rec_off = cword[cfirst[L]];
            sg.flags = kSegCluster;
            double cost = 0.0;
            for (int64_t j = 0; j < cc[L]; ++j) cost += ct[cfirst[L] + j];
            out.base.push_back(sg);
            out.unit_cost.push_back(cost / double(sg.n_pairs));
        }
        const int nb = meta.group_nuc_begin[g], ne = meta.group_nuc_end[g];
        if (out.base.size() == first_seg && ne > nb) {
            Segment sg{};
            sg.rec_off = base + ow + cw + mw;
            out.base.push_back(sg);
            out.unit_cost.push_back(0.0);
        }
        if (out.base.size() > first_seg) {
            out.base[first_seg].nuc_begin = nb;
            out.base[first_seg].nuc_end = ne;
            out.base.back().flags |= kSegEndGroup;
        }
        words += ow + cw + mw;
    }
    if (nC > 0 && words > int64_t(UINT32_MAX)) return ENV_E_UNSUPPORTED;  // member tables hold 32-bit words
    out.words = words;
    out.n_clusters = nC;
    out.n_members = mpos[nC];

    lap("group tables");
    // ---- 6. records and the density-fold tables
    uint32_t* rec = ar.alloc<uint32_t>(words);
    int64_t* d_ooff = ar.upload(ooff);
    UpdCluster* ucl = ar.alloc<UpdCluster>(nC);
    int64_t* members = ar.alloc<int64_t>(out.n_members);
    int64_t* moff = ar.alloc<int64_t>(out.n_members + 1);
    if (!rec || !d_ooff || !ucl || !members || !moff) return ENV_E_NOMEM;
    DB_CHECK(hipMemsetAsync(rec, 0, size_t(std::max<int64_t>(words, 1)) * 4, st) == hipSuccess);
    if (n_pairs > 0) {
        int32_t* f = ar.alloc<int32_t>(n_pairs);
        int32_t* orank = ar.alloc<int32_t>(n_pairs);
        if (!f || !orank) return ENV_E_NOMEM;
        DB_LAUNCH(n_pairs, k_not_in_cluster, in_cl, n_pairs, f);
        size_t ts = 0;
        DB_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, ts, f, orank, int(n_pairs), st) == hipSuccess);
        void* tmp = ar.alloc<char>(int64_t(ts));
        if (!tmp) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp, ts, f, orank, int(n_pairs), st) == hipSuccess);
        DB_LAUNCH(n_pairs, k_place_pairs, pL, pg, in_cl, orank, pstart, d_ooff, n_pairs, a.fp64, upd);
    }
    if (nC > 0) {
        int64_t* d_cword = ar.upload(cword);
        int64_t* d_mbase = ar.upload(mbase);
        int64_t* d_mpos = ar.upload(mpos);
        if (!d_cword || !d_mbase || !d_mpos) return ENV_E_NOMEM;
        DB_LAUNCH(nC, k_place_clusters, a.fp64, cl_run, rstart, cval_s, d_cword, d_mbase, d_mpos, nC, pL, pc, pr2,
                  upd, members, ucl, rec, words);
    }
    DB_LAUNCH(n_pairs, k_pair_records, upd, pc, pp, pr2, pL, n_pairs, a.fp64, rec, words);
    DB_CHECK(hipMemsetAsync(moff, 0, sizeof(int64_t), st) == hipSuccess);
    if (out.n_members > 0) {
        int64_t* sz = ar.alloc<int64_t>(out.n_members);
        if (!sz) return ENV_E_NOMEM;
        DB_LAUNCH(out.n_members, k_member_sizes, members, pL, out.n_members, sz);
        size_t ts = 0;
        DB_CHECK(hipcub::DeviceScan::InclusiveSum(nullptr, ts, sz, moff + 1, int(out.n_members), st) ==
                 hipSuccess);
        void* tmp = ar.alloc<char>(int64_t(ts));
        if (!tmp) return ENV_E_NOMEM;
        DB_CHECK(hipcub::DeviceScan::InclusiveSum(tmp, ts, sz, moff + 1, int(out.n_members), st) ==
                 hipSuccess);
        DB_CHECK(download1(&out.hm_words, moff + out.n_members, st));
    }
    DB_CHECK(hipStreamSynchronize(st) == hipSuccess);
    lap("records");
    out.d_rec = rec;
    out.d_pairs = upd;
    out.d_clusters = ucl;
    out.d_members = members;
    out.d_moff = moff;
    for (void* p : {static_cast<void*>(rec), static_cast<void*>(upd), static_cast<void*>(ucl),
                    static_cast<void*>(members), static_cast<void*>(moff)})
        ar.release(p);
    out.device_bytes = words * 4 + (n_pairs + n_drop) * int64_t(sizeof(UpdPair)) + nC * int64_t(sizeof(UpdCluster)) +
                       (2 * out.n_members + 1) * 8;
    return ENV_OK;
}

}  // namespace envpot
