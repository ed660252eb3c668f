// Incremental density update (env_potential_update_density): the host turns
// the new density matrix into per-block weights and the per-group neutral
// scale; the device refolds every record's D and h and the clusters' merged
// h in place (update.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "devbuild_internal.h"
#include "handle.h"
#include "update_internal.h"

namespace envpot {

namespace {

template <typename T>
env_status upload_vec(const std::vector<T>& v, T** dst, int64_t& bytes) {
    const size_t nb = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) return ENV_E_NOMEM;
    bytes += int64_t(nb);
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    return ENV_OK;
}

template <typename T>
env_status alloc_dev(size_t n, T** dst, int64_t& bytes) {
    const size_t nb = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) return ENV_E_NOMEM;
    bytes += int64_t(nb);
    return ENV_OK;
}

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

}  // namespace

void free_update_state(UpdateState* u) {
    if (!u) return;
    (void)hipFree(u->d_pairs);
    (void)hipFree(u->d_shells);
    (void)hipFree(u->d_blk);
    (void)hipFree(u->d_woff);
    (void)hipFree(u->d_moff);
    (void)hipFree(u->d_hm);
    (void)hipFree(u->d_exps);
    (void)hipFree(u->d_cnorm);
    (void)hipFree(u->d_W);
    (void)hipFree(u->d_scale);
    (void)hipFree(u->d_M);
    (void)hipFree(u->d_clusters);
    (void)hipFree(u->d_members);
    (void)hipFree(u->d_charge);
    (void)hipFree(u->d_shell_of_bf);
    (void)hipFree(u->d_bf0);
    (void)hipFree(u->d_shell_l);
    (void)hipFree(u->d_adj_begin);
    (void)hipFree(u->d_adj_J);
    (void)hipFree(u->d_adj_blk);
    (void)hipFree(u->d_adj_tr);
    (void)hipFree(u->d_cscale);
    (void)hipFree(u->d_Wd);
    (void)hipFree(u->d_Wt);
    (void)hipFree(u->d_err);
    (void)hipFree(u->d_gpb);
    (void)hipFree(u->d_dropb);
    (void)hipFree(u->d_gq);
    delete u;
}

namespace {

// The update tables that depend on the blocks and the basis only (both
// builds): shells, blocks, far-field matrices, block weights and the
// per-shell block lists; the caller attaches the pairs and clusters.
UpdateState* block_state(const PairList& pl, const PairSources& src, env_status* st) {
    const int n_shells = int(src.shell_l.size());
    std::vector<UpdShell> shells(n_shells);
    for (int s = 0; s < n_shells; ++s) {
        UpdShell& sh = shells[s];
        std::memset(&sh, 0, sizeof(sh));
        for (int c = 0; c < 3; ++c) sh.A[c] = src.atom_xyz[3 * size_t(src.shell_atom[s]) + c];
        sh.l = src.shell_l[s];
        sh.poff = src.poff[s];
        sh.noff = src.noff[s];
    }
    const int64_t n_blocks = int64_t(src.blk_I.size());
    std::vector<int32_t> blk(2 * size_t(n_blocks));
    for (int64_t b = 0; b < n_blocks; ++b) {
        blk[2 * b] = src.blk_I[b];
        blk[2 * b + 1] = src.blk_J[b];
    }
    // far-field matrices: column j of M_L is far_coefs of the unit vector e_j
    std::vector<double> M(kFarMatOff[kLMax + 1], 0.0);
    for (int L = 0; L <= kLMax; ++L) {
        const int nc = kNComp[L];
        double D[35], h[35];
        for (int j = 0; j < nc; ++j) {
            for (int k = 0; k < nc; ++k) D[k] = (k == j) ? 1.0 : 0.0;
            far_coefs(L, D, h);
            for (int i = 0; i < nc; ++i) M[kFarMatOff[L] + i * nc + j] = h[i];
        }
    }
    UpdateState* u = new (std::nothrow) UpdateState;
    if (!u) {
        *st = ENV_E_NOMEM;
        return nullptr;
    }
    u->n_groups = pl.n_groups;
    u->nbf = pl.nbf;
    u->n_shells = n_shells;
    u->neutralize = src.neutralize;
    u->shell_l = src.shell_l;
    u->bf0 = src.bf0;
    u->shell_of_bf.resize(pl.nbf);
    for (int s = 0; s < n_shells; ++s)
        for (int k = src.bf0[s]; k < src.bf0[s + 1]; ++k) u->shell_of_bf[k] = s;
    u->cscale = src.cscale;
    u->group_charge = src.group_charge;
    u->group_pair_begin = pl.group_pair_begin;
    u->n_blocks = n_blocks;
    u->blk_I = src.blk_I;
    u->blk_J = src.blk_J;
    // compact block weights: nI x nJ per block
    u->woff.assign(size_t(n_blocks) + 1, 0);
    for (int64_t b = 0; b < n_blocks; ++b)
        u->woff[b + 1] = u->woff[b] + ncart(src.shell_l[src.blk_I[b]]) * ncart(src.shell_l[src.blk_J[b]]);
    // per shell: its blocks by partner shell, ascending
    {
        std::vector<std::vector<std::pair<int32_t, int64_t>>> adj(n_shells);  // (partner, block*2 + transposed)
        for (int64_t b = 0; b < n_blocks; ++b) {
            adj[src.blk_I[b]].push_back({src.blk_J[b], 2 * b});
            if (src.blk_I[b] != src.blk_J[b]) adj[src.blk_J[b]].push_back({src.blk_I[b], 2 * b + 1});
        }
        u->adj_begin.assign(size_t(n_shells) + 1, 0);
        for (int sI = 0; sI < n_shells; ++sI) {
            std::sort(adj[sI].begin(), adj[sI].end());
            u->adj_begin[sI + 1] = u->adj_begin[sI] + int64_t(adj[sI].size());
            for (const auto& e : adj[sI]) {
                u->adj_J.push_back(e.first);
                u->adj_blk.push_back(int32_t(e.second >> 1));
                u->adj_tr.push_back(uint8_t(e.second & 1));
            }
        }
    }
    env_status s = upload_vec(shells, &u->d_shells, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(blk, &u->d_blk, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(src.exps, &u->d_exps, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(src.cnorm, &u->d_cnorm, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(M, &u->d_M, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->woff, &u->d_woff, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(u->woff.back()), &u->d_W, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(std::max(pl.n_groups, 1)), &u->d_scale, u->device_bytes);
    // the device parse of CSR densities: basis and block lists, element buffers
    if (s == ENV_OK) s = upload_vec(u->shell_of_bf, &u->d_shell_of_bf, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->bf0, &u->d_bf0, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->shell_l, &u->d_shell_l, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->adj_begin, &u->d_adj_begin, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->adj_J, &u->d_adj_J, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->adj_blk, &u->d_adj_blk, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->adj_tr, &u->d_adj_tr, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(u->cscale, &u->d_cscale, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(u->woff.back()), &u->d_Wd, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(u->woff.back()), &u->d_Wt, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(1), &u->d_err, u->device_bytes);
    if (s != ENV_OK) {
        free_update_state(u);
        *st = s;
        return nullptr;
    }
    return u;
}

// The group ranges of the per-group charge sums, once pairs and dropped
// pairs are attached.
env_status group_tables(UpdateState* u) {
    std::vector<int64_t> dropb(size_t(u->n_groups) + 1, 0);
    for (int64_t j = 0; j < int64_t(u->drop_group.size()); ++j) {
        const int32_t g = u->drop_group[j];
        if (g < 0 || g >= u->n_groups || (j > 0 && g < u->drop_group[j - 1])) return ENV_E_ARG;
        ++dropb[size_t(g) + 1];
    }
    for (int g = 0; g < u->n_groups; ++g) dropb[g + 1] += dropb[g];
    env_status s = upload_vec(u->group_pair_begin, &u->d_gpb, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(dropb, &u->d_dropb, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(2 * size_t(std::max(u->n_groups, 1)), &u->d_gq, u->device_bytes);
    return s;
}

}  // namespace

// Device tables of the update (on the current device) for a host-packed
// pair list.  Returns nullptr when the input does not fit them (then
// updates are unsupported).
UpdateState* make_update_state(const PairList& pl, const PairSources& src, const LayoutMap& map,
                               env_status* st) {
    *st = ENV_OK;
    const int64_t n_pairs = int64_t(pl.L.size());
    const int64_t n_drop = src.neutralize ? int64_t(src.drop_blk.size()) : 0;
    if (int64_t(src.pair_blk.size()) != n_pairs || int64_t(map.pair_word.size()) != n_pairs) return nullptr;
    std::vector<UpdPair> pairs(size_t(n_pairs + n_drop));
    for (int64_t k = 0; k < n_pairs; ++k) {
        if (src.pair_ia[k] > 32767 || src.pair_ib[k] > 32767 || map.pair_word[k] < 0) return nullptr;
        UpdPair& q = pairs[k];
        q.blk = src.pair_blk[k];
        q.ia = int16_t(src.pair_ia[k]);
        q.ib = int16_t(src.pair_ib[k]);
        q.group = pl.group[k];
        q.L = pl.L[k];
        q.word = map.pair_word[k];
    }
    for (int64_t j = 0; j < n_drop; ++j) {
        if (src.drop_ia[j] > 32767 || src.drop_ib[j] > 32767) return nullptr;
        UpdPair& q = pairs[n_pairs + j];
        q.blk = src.drop_blk[j];
        q.ia = int16_t(src.drop_ia[j]);
        q.ib = int16_t(src.drop_ib[j]);
        q.group = src.drop_group[j];
        q.L = 0;
        q.word = -1;
    }
    const int64_t n_clusters = int64_t(map.cl_word.size());
    std::vector<UpdCluster> cl(static_cast<size_t>(n_clusters));
    for (int64_t c = 0; c < n_clusters; ++c) {
        cl[c].word = map.cl_word[c];
        cl[c].begin = map.cl_begin[c];
        cl[c].end = map.cl_begin[c + 1];
        cl[c].L = map.cl_L[c];
        cl[c].pad = 0;
    }
    std::vector<int64_t> moff(map.cl_members.size() + 1, 0);
    for (size_t m = 0; m < map.cl_members.size(); ++m) moff[m + 1] = moff[m] + kNComp[pl.L[map.cl_members[m]]];
    UpdateState* u = block_state(pl, src, st);
    if (!u) return nullptr;
    u->n_pairs = n_pairs;
    u->n_drop = n_drop;
    u->n_clusters = n_clusters;
    u->n_members = int64_t(map.cl_members.size());
    u->drop_group.assign(src.drop_group.begin(), src.drop_group.begin() + n_drop);
    env_status s = upload_vec(pairs, &u->d_pairs, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(cl, &u->d_clusters, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(map.cl_members, &u->d_members, u->device_bytes);
    if (s == ENV_OK) s = upload_vec(moff, &u->d_moff, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(moff.back()), &u->d_hm, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(n_pairs + n_drop), &u->d_charge, u->device_bytes);
    if (s == ENV_OK) s = group_tables(u);
    if (s != ENV_OK) {
        free_update_state(u);
        *st = s;
        return nullptr;
    }
    return u;
}

// The same tables for a device-built pair list: the pair, cluster and member
// tables the device build wrote are taken over (db's pointers are cleared).
UpdateState* make_update_state_device(const PairList& meta, const PairSources& src, DevBuild& db,
                                      env_status* st) {
    *st = ENV_OK;
    UpdateState* u = block_state(meta, src, st);
    if (!u) return nullptr;
    u->n_pairs = db.n_pairs;
    u->n_drop = db.n_drop;
    u->n_clusters = db.n_clusters;
    u->n_members = db.n_members;
    u->drop_group = db.drop_group;
    u->d_pairs = db.d_pairs;
    u->d_clusters = db.d_clusters;
    u->d_members = db.d_members;
    u->d_moff = db.d_moff;
    db.d_pairs = nullptr;
    db.d_clusters = nullptr;
    db.d_members = nullptr;
    db.d_moff = nullptr;
    u->device_bytes += (db.n_pairs + db.n_drop) * int64_t(sizeof(UpdPair)) +
                       db.n_clusters * int64_t(sizeof(UpdCluster)) + (2 * db.n_members + 1) * 8;
    env_status s = alloc_dev(size_t(db.hm_words), &u->d_hm, u->device_bytes);
    if (s == ENV_OK) s = alloc_dev(size_t(db.n_pairs + db.n_drop), &u->d_charge, u->device_bytes);
    if (s == ENV_OK) s = group_tables(u);
    if (s != ENV_OK) {
        free_update_state(u);
        *st = s;
        return nullptr;
    }
    return u;
}

}  // namespace envpot

using namespace envpot;

extern "C" {

env_status env_potential_update_density(env_potential* h, const env_density* P, void* stream) {
    if (!h || !P) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    UpdateState* u = h->upd;
    if (!u) return ENV_E_UNSUPPORTED;
    const int nbf = u->nbf;
    if (P->nbf != nbf) return ENV_E_ARG;
    if (P->format != ENV_DENSITY_DENSE && P->format != ENV_DENSITY_CSR) return ENV_E_ARG;
    if (nbf > 0 && !P->values) return ENV_E_ARG;
    if (P->format == ENV_DENSITY_CSR && (!P->row_ptr || (nbf > 0 && !P->col))) return ENV_E_ARG;
    const char* tenv = std::getenv("ENVPOT_TIMING");
    const bool timing = tenv && *tenv && *tenv != '0';
    auto tlast = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
        if (!timing) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[envpot update] %-22s %8.3f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - tlast).count());
        tlast = now;
    };
    DeviceGuard g(h->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // a CSR density is parsed on the device (ENVPOT_HOST_PARSE=1: on the
    // host, as a dense one always is); both give the same weights W
    const char* hpe = std::getenv("ENVPOT_HOST_PARSE");
    const bool dev_parse = P->format == ENV_DENSITY_CSR && nbf > 0 && u->d_Wd && !(hpe && *hpe && *hpe != '0');
    std::vector<double> W;
    if (dev_parse) {
        if (P->row_ptr[0] != 0) return ENV_E_ARG;
        for (int mu = 0; mu < nbf; ++mu)
            if (P->row_ptr[mu + 1] < P->row_ptr[mu]) return ENV_E_ARG;
        const int64_t nnz = P->row_ptr[nbf];
        const int64_t nw = u->woff.back();
        int64_t* d_rp = nullptr;
        int32_t* d_col = nullptr;
        double* d_val = nullptr;
        env_status pst = ENV_OK;
        if (hipMallocAsync(reinterpret_cast<void**>(&d_rp), size_t(nbf + 1) * sizeof(int64_t), st) != hipSuccess ||
            hipMallocAsync(reinterpret_cast<void**>(&d_col), size_t(std::max<int64_t>(nnz, 1)) * sizeof(int32_t),
                           st) != hipSuccess ||
            hipMallocAsync(reinterpret_cast<void**>(&d_val), size_t(std::max<int64_t>(nnz, 1)) * sizeof(double),
                           st) != hipSuccess)
            pst = ENV_E_NOMEM;
        int32_t herr = 0;
        if (pst == ENV_OK &&
            (hipMemcpyAsync(d_rp, P->row_ptr, size_t(nbf + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
                 hipSuccess ||
             (nnz > 0 && hipMemcpyAsync(d_col, P->col, size_t(nnz) * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
                             hipSuccess) ||
             (nnz > 0 && hipMemcpyAsync(d_val, P->values, size_t(nnz) * sizeof(double), hipMemcpyHostToDevice,
                                        st) != hipSuccess) ||
             (nw > 0 && (hipMemsetAsync(u->d_Wd, 0, size_t(nw) * sizeof(double), st) != hipSuccess ||
                         hipMemsetAsync(u->d_Wt, 0, size_t(nw) * sizeof(double), st) != hipSuccess)) ||
             hipMemsetAsync(u->d_err, 0, sizeof(int32_t), st) != hipSuccess))
            pst = ENV_E_DEVICE;
        if (pst == ENV_OK) {
            ParseArgs pa{};
            pa.row_ptr = d_rp;
            pa.col = d_col;
            pa.val = d_val;
            pa.nnz = nnz;
            pa.nbf = nbf;
            pa.shell_of_bf = u->d_shell_of_bf;
            pa.bf0 = u->d_bf0;
            pa.shell_l = u->d_shell_l;
            pa.adj_begin = u->d_adj_begin;
            pa.adj_J = u->d_adj_J;
            pa.adj_blk = u->d_adj_blk;
            pa.adj_tr = u->d_adj_tr;
            pa.blk = u->d_blk;
            pa.woff = u->d_woff;
            pa.n_blocks = u->n_blocks;
            pa.cscale = u->d_cscale;
            pa.Wd = u->d_Wd;
            pa.Wt = u->d_Wt;
            pa.W = u->d_W;
            pa.err = u->d_err;
            if (launch_parse_csr(pa, stream) != 0 || launch_block_weights(pa, nw, stream) != 0 ||
                hipMemcpyAsync(&herr, u->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
                pst = ENV_E_DEVICE;
        }
        (void)hipFreeAsync(d_rp, st);
        (void)hipFreeAsync(d_col, st);
        (void)hipFreeAsync(d_val, st);
        if (hipStreamSynchronize(st) != hipSuccess && pst == ENV_OK) pst = ENV_E_DEVICE;
        if (pst != ENV_OK) return pst;
        if (herr != 0) return ENV_E_ARG;  // the records are untouched: only W was written
        lap("device parse");
    } else {
        // weights of the known blocks, written through each shell's block list
        // (columns ascending: one step per element; unsorted columns restart the
        // walk); an element of an unknown block makes the density invalid
        std::vector<double> Wd(size_t(u->woff.back()), 0.0), Wt(size_t(u->woff.back()), 0.0);
        auto row = [&](int mu, auto&& next) -> env_status {
            const int I = u->shell_of_bf[mu], x = mu - u->bf0[I];
            const int64_t a0 = u->adj_begin[I], a1 = u->adj_begin[I + 1];
            int64_t ptr = a0;
            int nu, prev = -1;
            double v;
            while (next(nu, v)) {
                if (!std::isfinite(v)) return ENV_E_ARG;
                if (v == 0.0) continue;
                const int J = u->shell_of_bf[nu], y = nu - u->bf0[J];
                if (nu < prev) ptr = a0;
                prev = nu;
                while (ptr < a1 && u->adj_J[ptr] < J) ++ptr;
                if (ptr == a1 || u->adj_J[ptr] != J) return ENV_E_ARG;  // a block the build did not see
                const int32_t b = u->adj_blk[ptr];
                const int nJb = ncart(u->shell_l[u->blk_J[b]]);
                if (u->adj_tr[ptr]) Wt[u->woff[b] + y * nJb + x] += v;  // element (J, I) of block (I, J)
                else Wd[u->woff[b] + x * nJb + y] += v;
            }
            return ENV_OK;
        };
        if (P->format == ENV_DENSITY_DENSE) {
            for (int mu = 0; mu < nbf; ++mu) {
                int nu = 0;
                const double* rowv = P->values + size_t(mu) * nbf;
                const env_status r = row(mu, [&](int& c, double& v) {
                    if (nu >= nbf) return false;
                    c = nu;
                    v = rowv[nu++];
                    return true;
                });
                if (r != ENV_OK) return r;
            }
        } else {
            if (P->row_ptr[0] != 0) return ENV_E_ARG;
            for (int mu = 0; mu < nbf; ++mu) {
                if (P->row_ptr[mu + 1] < P->row_ptr[mu]) return ENV_E_ARG;
                int64_t k = P->row_ptr[mu];
                const int64_t ke = P->row_ptr[mu + 1];
                bool bad = false;
                const env_status r = row(mu, [&](int& c, double& v) {
                    if (k >= ke) return false;
                    c = P->col[k];
                    v = P->values[k++];
                    if (c < 0 || c >= nbf) {
                        bad = true;
                        return false;
                    }
                    return true;
                });
                if (bad) return ENV_E_ARG;
                if (r != ENV_OK) return r;
            }
        }
        lap("density blocks");
        // symmetry (block (J, I) is the transpose of (I, J)), then the weights
        // f P_xy s_x s_y with f = 2 off the diagonal blocks
        W.assign(size_t(u->woff.back()), 0.0);
        for (int64_t b = 0; b < u->n_blocks; ++b) {
            const int I = u->blk_I[b], J = u->blk_J[b];
            const int nI = ncart(u->shell_l[I]), nJ = ncart(u->shell_l[J]);
            const double* a = &Wd[u->woff[b]];
            const double* t = &Wt[u->woff[b]];
            for (int x = 0; x < nI; ++x)
                for (int y = 0; y < nJ; ++y) {
                    const double p = a[x * nJ + y], q = (I == J) ? a[y * nJ + x] : t[x * nJ + y];
                    if (std::fabs(p - q) > 1e-10 * (std::fabs(p) + std::fabs(q))) return ENV_E_ARG;
                }
            const double f = (I == J) ? 1.0 : 2.0;
            double* w = &W[u->woff[b]];
            for (int x = 0; x < nI; ++x)
                for (int y = 0; y < nJ; ++y)
                    w[x * nJ + y] = f * a[x * nJ + y] * u->cscale[u->bf0[I] + x] * u->cscale[u->bf0[J] + y];
        }
        lap("block weights");
    }
    UpdateArgs A{};
    A.pairs = u->d_pairs;
    A.n_pairs = u->n_pairs;
    A.n_drop = u->n_drop;
    A.shells = u->d_shells;
    A.blk = u->d_blk;
    A.woff = u->d_woff;
    A.exps = u->d_exps;
    A.cnorm = u->d_cnorm;
    A.W = u->d_W;
    A.scale = u->d_scale;
    A.M = u->d_M;
    A.clusters = u->d_clusters;
    A.members = u->d_members;
    A.moff = u->d_moff;
    A.hm = u->d_hm;
    A.n_members = int64_t(u->n_members);
    A.n_clusters = u->n_clusters;
    A.rec = h->d_rec;
    A.charge = u->d_charge;
    A.fp64 = h->precision == ENV_PREC_FP64 ? 1 : 0;
    // host buffers below are read or written by copies on `st`: every exit
    // waits for the stream first
    auto fail = [&]() {
        (void)hipStreamSynchronize(st);
        return ENV_E_DEVICE;
    };
    if (!W.empty() && hipMemcpyAsync(u->d_W, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
                          hipSuccess)
        return fail();
    // electron counts per group; with ENV_NEUTRALIZE the scale to the group's
    // nuclear charge (screened-out pairs included, as at create)
    // (the charges of every pair, summed per group on the device in fixed order)
    std::vector<double> gq(2 * size_t(u->n_groups), 0.0);
    if (launch_update_charges(A, stream) != 0) return fail();
    if (u->n_groups > 0 &&
        (launch_group_charges(u->d_charge, u->d_gpb, u->d_dropb, u->n_pairs, u->n_groups, u->d_gq, stream) != 0 ||
         hipMemcpyAsync(gq.data(), u->d_gq, gq.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess))
        return fail();
    if (hipStreamSynchronize(st) != hipSuccess) return ENV_E_DEVICE;
    lap("upload, charges");
    std::vector<double> qkept(u->n_groups, 0.0), qall(u->n_groups, 0.0), scale(std::max(u->n_groups, 1), 1.0);
    double electrons = 0.0;
    for (int gi = 0; gi < u->n_groups; ++gi) {
        qkept[gi] = gq[2 * size_t(gi)];
        qall[gi] = gq[2 * size_t(gi) + 1] + qkept[gi];
        if (u->neutralize && qall[gi] != 0.0) scale[gi] = u->group_charge[gi] / qall[gi];
        electrons += scale[gi] * qkept[gi];
    }
    if (hipMemcpyAsync(u->d_scale, scale.data(), scale.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return fail();
    // from here on the records change: anything derived from the old density
    // (a trained surrogate) is out of date, even if a launch below fails
    ++h->density_gen;
    if (launch_update_pairs(A, stream) != 0) return fail();
    if (launch_update_members(A, stream) != 0) return fail();
    if (launch_update_clusters(A, stream) != 0) return fail();
    if (hipStreamSynchronize(st) != hipSuccess) return ENV_E_DEVICE;
    lap("scale, records");
    h->info.electrons = electrons;
    return ENV_OK;
}

}  // extern "C"
