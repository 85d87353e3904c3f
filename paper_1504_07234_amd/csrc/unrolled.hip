// K unrolled iterations of eq. (MLBA2) and their reverse-mode gradient with
// respect to the per-band thresholds mu, the Tikhonov parameter alpha, the
// PSF and the observation (rectangular blur of section 2.1, BCCB
// preconditioner of Algorithm 1), for a batch of images advanced together:
// every phase is one launch over the tiles of all images, as in the batched
// restoration.
//
// Forward:  z_0 = 0;  u_k = W^T(delta S_mu(z_k)),  r_k = g - A u_k,
//           t_k = P_alpha r_k,  z_{k+1} = z_k + W A^T t_k;  f = W^T(delta S_mu(z_K)),
// keeping z at k = 0, c, 2c, ... (caller-owned checkpoints).
//
// Reverse (loss l with cotangent fbar = dl/df): zbar_K = delta D_K W fbar,
// then for k = K-1 .. 0, with D_k = diag(1{|z_k| > mu}):
//   wbar = W^T zbar,  tbar = A wbar,  rbar = P tbar,  v = W A^T rbar,
//   dmu_b += delta <v, sgn(z_k) D_k>_b,  dalpha -= <rbar, t_k>,  dg += rbar,
//   dH += corr(wbar, t_k) - corr(u_k, rbar) + (spectral term through P),
//   zbar -= delta D_k v;
// and dmu_b -= delta <W fbar, sgn(z_K) D_K>_b for the output's own threshold.
// The soft threshold is differentiated almost everywhere: dS/dz = 1{|z| > mu},
// dS/dmu = -sgn(z) 1{|z| > mu}, both taken as 0 at the kink |z| = mu.  delta
// is a constant.  Each checkpoint segment is recomputed once, keeping its
// states z_k, u_k, t_k and the filtered spectra of t_k.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "mlba.h"
#include "plan.hpp"

using namespace mlba;

namespace {

struct Map {
    int nblocks = 0;
    int* bmap = nullptr;
    int* bfirst = nullptr;
};

struct ImgBufs {
    float* zs = nullptr;     // c states [c][bands][N][N]: z_{jc+1} .. z_{jc+c}
    float* U = nullptr;      // [c][N][N]
    float* Tk = nullptr;     // [c][n][n]
    float2* Sk = nullptr;    // [c][n/2+1][n]
    float* zbar = nullptr;   // [bands][N][N]
    float* wbar = nullptr;   // [N][N]
    float* zK = nullptr;     // final forward state [bands][N][N]
    float* eacc = nullptr;   // [n/2+1][n]
};

}  // namespace

struct mlba_unrolled_s {
    int count = 0, levels = 0, bands = 0, p = 0, iters = 0, ce = 0, J = 0, nmax = 8;
    int any_len = 0;  // some image's transform takes the Bluestein form
    std::vector<mlba_plan_t> plans;
    std::vector<BatchImage> base;
    std::vector<ImgBufs> bufs;
    std::vector<void*> allocs;
    int* maps = nullptr;
    Map conv_a, conv_at, pre[3], syn[5], ana[5], adj[5], corr, fill;
    double* dblock = nullptr;  // running partials (doubles), zeroed per backward
    size_t dcount = 0;
    float* eblock = nullptr;   // eacc of every image, zeroed per backward
    size_t ecount = 0;
    double* mu_part[4] = {nullptr, nullptr, nullptr, nullptr};
    double* alpha_part = nullptr;
    double* corr_part = nullptr;
    double* spec = nullptr;
    BatchImage* tables = nullptr;  // device descriptor tables
    int table_cap = 0;             // tables of `count` descriptors
    std::vector<BatchImage> host_tables;
    hipEvent_t done = nullptr;  // recorded after every call that enqueues work
};

namespace {

void destroy_unrolled(mlba_unrolled_s* U) {
    if (U->done) hipEventDestroy(U->done);
    for (void* a : U->allocs) hipFree(a);
    delete U;
}

// The object's and its plans' completion events on s (their buffers were used).
int note_unrolled(mlba_unrolled_s* U, hipStream_t s) {
    HIPCHK(hipEventRecord(U->done, s));
    for (mlba_plan_t P : U->plans)
        if (P->done) HIPCHK(hipEventRecord(P->done, s));
    return MLBA_OK;
}

int ualloc(mlba_unrolled_s* U, void** ptr, size_t bytes) {
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        *ptr = nullptr;
        return MLBA_ENOMEM;
    }
    U->allocs.push_back(*ptr);
    return MLBA_OK;
}

template <class T>
int ualloc_t(mlba_unrolled_s* U, T** ptr, size_t count) {
    void* v = nullptr;
    const int st = ualloc(U, &v, count * sizeof(T));
    *ptr = (T*)v;
    return st;
}

void build_map(const std::vector<int>& tiles, std::vector<int>& hm, std::vector<size_t>& offs, Map& m) {
    m.nblocks = 0;
    for (int t : tiles) m.nblocks += t;
    offs.push_back(hm.size());
    for (size_t i = 0; i < tiles.size(); ++i)
        for (int t = 0; t < tiles[i]; ++t) hm.push_back((int)i);
    offs.push_back(hm.size());
    int acc = 0;
    for (int t : tiles) {
        hm.push_back(acc);
        acc += t;
    }
}

size_t state_elems(const BatchImage& b) { return (size_t)b.bands * b.N * b.N; }
size_t spec_elems(const BatchImage& b) { return (size_t)(b.n / 2 + 1) * b.n; }

// segment j covers iterations [j*ce, j*ce + seg_len(j))
int seg_len(const mlba_unrolled_s* U, int j) { return std::min(U->ce, U->iters - j * U->ce); }

// One forward iteration with descriptor table T.
int enqueue_step(const mlba_unrolled_s* U, const BatchImage* T, hipStream_t s) {
    for (int lev = U->levels; lev >= 1; --lev) {
        const Map& m = U->syn[lev];
        HIPCHK(launch_synthesis_batched(T, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 0, s));
    }
    HIPCHK(launch_conv_batched(T, U->conv_a.bmap, U->conv_a.bfirst, U->conv_a.nblocks, 1, U->p, nullptr, s));
    for (int pass = 0; pass < 3; ++pass)
        HIPCHK(launch_precond_batched(T, U->pre[pass].bmap, U->pre[pass].bfirst, U->pre[pass].nblocks, pass,
                                      MLBA_PRECOND_BCCB, U->nmax, s, U->any_len));
    HIPCHK(launch_conv_batched(T, U->conv_at.bmap, U->conv_at.bfirst, U->conv_at.nblocks, 0, U->p, nullptr, s));
    for (int lev = 1; lev <= U->levels; ++lev) {
        const Map& m = U->ana[lev];
        HIPCHK(launch_analysis_batched(T, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), s));
    }
    return MLBA_OK;
}

// Validates the per-call scalars and fills alpha, delta and mu of the base descriptors.
int set_params(mlba_unrolled_s* U, double alpha, const double* mu, int n_mu, double delta) {
    if (!(alpha > 0.0) || !isfinite(alpha) || !(delta > 0.0) || !isfinite(delta)) return MLBA_EINVAL;
    if (!mu || (n_mu != 1 && n_mu != U->bands)) return MLBA_EINVAL;
    for (int b = 0; b < U->bands; ++b) {
        const double m = mu[n_mu == 1 ? 0 : b];
        if (!(m >= 0.0) || !isfinite(m)) return MLBA_EINVAL;
    }
    for (BatchImage& d : U->base) {
        d.alpha = (float)alpha;
        d.delta = (float)delta;
        for (int b = 0; b < U->bands; ++b) d.mu[b] = (float)mu[n_mu == 1 ? 0 : b];
    }
    return MLBA_OK;
}

// Appends one table (a copy of the base descriptors edited by `edit`) and
// returns its index.
template <class F>
int add_table(mlba_unrolled_s* U, F edit) {
    const int idx = (int)(U->host_tables.size() / U->count);
    for (int i = 0; i < U->count; ++i) {
        BatchImage d = U->base[i];
        edit(i, d);
        U->host_tables.push_back(d);
    }
    return idx;
}

int upload_tables(mlba_unrolled_s* U, hipStream_t s) {
    const int n = (int)(U->host_tables.size() / U->count);
    if (n > U->table_cap) return MLBA_EINVAL;  // sized at creation; not reached
    HIPCHK(hipMemcpyAsync(U->tables, U->host_tables.data(), U->host_tables.size() * sizeof(BatchImage),
                          hipMemcpyHostToDevice, s));
    return MLBA_OK;
}

const BatchImage* table(const mlba_unrolled_s* U, int idx) { return U->tables + (size_t)idx * U->count; }

float* ckpt_slot(float* const* ckpt, const mlba_unrolled_s* U, int i, int j) {
    return ckpt[i] + (size_t)j * state_elems(U->base[i]);
}

}  // namespace

extern "C" {

int mlba_unrolled_create(mlba_unrolled_t* out, int count, const mlba_plan_t* plans, int iters, int ckpt_every,
                         hipStream_t s) {
    if (!out || !plans || count < 1 || iters < 1 || ckpt_every < 1 || ckpt_every > iters) return MLBA_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return MLBA_EINVAL;
        if (plans[i]->bc != MLBA_BC_RECT || plans[i]->precond != MLBA_PRECOND_BCCB) return MLBA_EUNSUPPORTED;
        if (plans[i]->levels != plans[0]->levels || plans[i]->p != plans[0]->p) return MLBA_EINVAL;
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return MLBA_EINVAL;
    }
    mlba_unrolled_s* U = new (std::nothrow) mlba_unrolled_s();
    if (!U) return MLBA_ENOMEM;
    U->count = count;
    U->levels = plans[0]->levels;
    U->bands = plans[0]->bands;
    U->p = plans[0]->p;
    U->iters = iters;
    U->ce = ckpt_every;
    U->J = (iters + ckpt_every - 1) / ckpt_every;
    U->plans.assign(plans, plans + count);
    U->base.resize(count);
    U->bufs.resize(count);
    for (int i = 0; i < count; ++i) {
        U->base[i] = plan_desc(plans[i]);
        U->nmax = std::max(U->nmax, plans[i]->n);
        if (plans[i]->fd.m > 0) U->any_len = 1;  // a Bluestein-form transform
    }
    int st = MLBA_OK;
#define UALLOC(ptr, cnt)                  \
    do {                                  \
        st = ualloc_t(U, &(ptr), (cnt));  \
        if (st) {                         \
            destroy_unrolled(U);          \
            return st;                    \
        }                                 \
    } while (0)
    const int c = U->ce;
    for (int i = 0; i < count; ++i) {
        const BatchImage& b = U->base[i];
        ImgBufs& q = U->bufs[i];
        const size_t NN = (size_t)b.N * b.N, nn = (size_t)b.n * b.n;
        UALLOC(q.zs, (size_t)c * state_elems(b));
        UALLOC(q.U, (size_t)c * NN);
        UALLOC(q.Tk, (size_t)c * nn);
        UALLOC(q.Sk, (size_t)c * spec_elems(b));
        UALLOC(q.zbar, state_elems(b));
        UALLOC(q.wbar, NN);
        UALLOC(q.zK, state_elems(b));
    }
    // phase maps
    std::vector<int> hm;
    std::vector<size_t> offs;
    std::vector<Map*> order;
    std::vector<int> t(count);
    auto add = [&](Map& m) {
        build_map(t, hm, offs, m);
        order.push_back(&m);
    };
    for (int i = 0; i < count; ++i) t[i] = conv_batched_tiles(U->base[i], 1);
    add(U->conv_a);
    for (int i = 0; i < count; ++i) t[i] = conv_batched_tiles(U->base[i], 0);
    add(U->conv_at);
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < count; ++i) t[i] = precond_pass_tiles(U->base[i], pass);
        add(U->pre[pass]);
    }
    for (int lev = 1; lev <= U->levels; ++lev) {
        for (int i = 0; i < count; ++i) t[i] = synthesis_level_tiles(U->base[i].N, 1 << (lev - 1));
        add(U->syn[lev]);
        for (int i = 0; i < count; ++i) t[i] = analysis_level_tiles(U->base[i].N, 1 << (lev - 1));
        add(U->ana[lev]);
        for (int i = 0; i < count; ++i) t[i] = analysis_adjoint_tiles(U->base[i].N, 1 << (lev - 1));
        add(U->adj[lev]);
    }
    for (int i = 0; i < count; ++i) t[i] = psf_corr_tiles(U->base[i]);
    add(U->corr);
    for (int i = 0; i < count; ++i) t[i] = fill_tiles(U->base[i]);
    add(U->fill);
    UALLOC(U->maps, hm.size());
    for (size_t q = 0; q < order.size(); ++q) {
        order[q]->bmap = U->maps + offs[2 * q];
        order[q]->bfirst = U->maps + offs[2 * q + 1];
    }
    // running partials
    const int pp = U->p * U->p;
    size_t off[7] = {0};
    U->dcount = 0;
    for (int lev = 1; lev <= U->levels; ++lev) {
        off[lev - 1] = U->dcount;
        U->dcount += (size_t)U->adj[lev].nblocks * 9;
    }
    off[4] = U->dcount;
    U->dcount += U->corr.nblocks;
    off[5] = U->dcount;
    U->dcount += (size_t)U->corr.nblocks * pp;
    off[6] = U->dcount;
    U->dcount += (size_t)count * pp;
    UALLOC(U->dblock, U->dcount);
    for (int lev = 1; lev <= U->levels; ++lev) U->mu_part[lev - 1] = U->dblock + off[lev - 1];
    U->alpha_part = U->dblock + off[4];
    U->corr_part = U->dblock + off[5];
    U->spec = U->dblock + off[6];
    U->ecount = 0;
    for (int i = 0; i < count; ++i) U->ecount += spec_elems(U->base[i]);
    UALLOC(U->eblock, U->ecount);
    size_t eo = 0;
    for (int i = 0; i < count; ++i) {
        U->bufs[i].eacc = U->eblock + eo;
        eo += spec_elems(U->base[i]);
    }
    // descriptor tables: forward 2J + 2, backward 2K + 2
    U->table_cap = std::max(2 * U->J + 2, 2 * iters + 2);
    UALLOC(U->tables, (size_t)U->table_cap * count);
#undef UALLOC
    hipError_t e = hipMemcpyAsync(U->maps, hm.data(), hm.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&U->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        destroy_unrolled(U);
        return MLBA_EHIP;
    }
    *out = U;
    return MLBA_OK;
}

int mlba_unrolled_destroy(mlba_unrolled_t U) {
    if (!U) return MLBA_EINVAL;
    if (U->done) (void)hipEventSynchronize(U->done);  // the object's last enqueued work
    destroy_unrolled(U);
    return MLBA_OK;
}

int mlba_unrolled_dims(mlba_unrolled_t U, int* segments, size_t* ckpt_elems_per_image) {
    if (!U) return MLBA_EINVAL;
    if (segments) *segments = U->J;
    if (ckpt_elems_per_image)
        for (int i = 0; i < U->count; ++i) ckpt_elems_per_image[i] = (size_t)U->J * state_elems(U->base[i]);
    return MLBA_OK;
}

int mlba_unrolled_forward(mlba_unrolled_t U, const float* const* g, double alpha, const double* mu, int n_mu,
                          double delta, float* const* ckpt, float* const* f, hipStream_t s) {
    if (!U || !g || !ckpt || !f) return MLBA_EINVAL;
    for (int i = 0; i < U->count; ++i)
        if (!g[i] || !ckpt[i] || !f[i]) return MLBA_EINVAL;
    STCHK(set_params(U, alpha, mu, n_mu, delta));
    U->host_tables.clear();
    const int J = U->J;
    // state written by segment j: the next checkpoint, or zK after the last one
    auto next_state = [&](int i, int j) { return j + 1 < J ? ckpt_slot(ckpt, U, i, j + 1) : U->bufs[i].zK; };
    const int t_fill = add_table(U, [&](int i, BatchImage& d) { d.z = ckpt_slot(ckpt, U, i, 0); });
    std::vector<int> t_first(J), t_rest(J);
    for (int j = 0; j < J; ++j) {
        t_first[j] = add_table(U, [&](int i, BatchImage& d) {
            d.g = g[i];
            d.zin = ckpt_slot(ckpt, U, i, j);
            d.z = next_state(i, j);
        });
        t_rest[j] = add_table(U, [&](int i, BatchImage& d) {
            d.g = g[i];
            d.zin = d.z = next_state(i, j);
        });
    }
    const int t_out = add_table(U, [&](int i, BatchImage& d) {
        d.zin = U->bufs[i].zK;
        d.f = f[i];
    });
    STCHK(upload_tables(U, s));
    HIPCHK(launch_fill_batched(table(U, t_fill), U->fill.bmap, U->fill.bfirst, U->fill.nblocks, s));
    for (int j = 0; j < J; ++j)
        for (int k = 0; k < seg_len(U, j); ++k) STCHK(enqueue_step(U, table(U, k == 0 ? t_first[j] : t_rest[j]), s));
    for (int lev = U->levels; lev >= 1; --lev) {
        const Map& m = U->syn[lev];
        HIPCHK(launch_synthesis_batched(table(U, t_out), m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 1, s));
    }
    return note_unrolled(U, s);
}

int mlba_unrolled_backward(mlba_unrolled_t U, const float* const* g, double alpha, const double* mu, int n_mu,
                           double delta, float* const* ckpt, const float* const* df, double* dmu, double* dalpha,
                           double* dpsf, float* const* dg, hipStream_t s) {
    if (!U || !g || !ckpt || !df || !dmu || !dalpha || !dpsf) return MLBA_EINVAL;
    for (int i = 0; i < U->count; ++i)
        if (!g[i] || !ckpt[i] || !df[i]) return MLBA_EINVAL;
    STCHK(set_params(U, alpha, mu, n_mu, delta));
    U->host_tables.clear();
    const int J = U->J;
    // z_k for k = j*ce + i: the checkpoint at i = 0, else recomputed slot i
    auto state = [&](int i, int j, int k) -> float* {
        return k == 0 ? ckpt_slot(ckpt, U, i, j) : U->bufs[i].zs + (size_t)(k - 1) * state_elems(U->base[i]);
    };
    std::vector<std::vector<int>> t_rec(J), t_adj(J);
    for (int j = 0; j < J; ++j) {
        const int L = seg_len(U, j);
        t_rec[j].resize(L);
        t_adj[j].resize(L);
        for (int k = 0; k < L; ++k) {
            t_rec[j][k] = add_table(U, [&](int i, BatchImage& d) {
                const ImgBufs& q = U->bufs[i];
                const BatchImage& b = U->base[i];
                d.g = g[i];
                d.zin = state(i, j, k);
                d.z = state(i, j, k + 1);
                d.u = q.U + (size_t)k * b.N * b.N;
                d.t = q.Tk + (size_t)k * b.n * b.n;
                d.sstore = q.Sk + (size_t)k * spec_elems(b);
            });
            t_adj[j][k] = add_table(U, [&](int i, BatchImage& d) {
                const ImgBufs& q = U->bufs[i];
                const BatchImage& b = U->base[i];
                d.g = nullptr;  // A wbar without the observation
                d.zin = q.zbar;
                d.u = q.wbar;
                d.sfwd = q.Sk + (size_t)k * spec_elems(b);
                d.eacc = q.eacc;
                d.zk = state(i, j, k);
                d.zbar = q.zbar;
                d.tk = q.Tk + (size_t)k * b.n * b.n;
                d.uk = q.U + (size_t)k * b.N * b.N;
                d.dg = dg ? dg[i] : nullptr;
            });
        }
    }
    const int t_init = add_table(U, [&](int i, BatchImage& d) {
        d.w = const_cast<float*>(df[i]);
        d.zk = state(i, J - 1, seg_len(U, J - 1));
        d.zbar = U->bufs[i].zbar;
    });
    const int t_end = add_table(U, [&](int i, BatchImage& d) { d.eacc = U->bufs[i].eacc; });
    STCHK(upload_tables(U, s));

    HIPCHK(launch_fill((float*)U->dblock, U->dcount * 2, 0.0f, s));
    HIPCHK(launch_fill(U->eblock, U->ecount, 0.0f, s));
    bool first = true;
    for (int j = J - 1; j >= 0; --j) {
        const int L = seg_len(U, j);
        for (int k = 0; k < L; ++k) STCHK(enqueue_step(U, table(U, t_rec[j][k]), s));
        if (j == J - 1)
            for (int lev = 1; lev <= U->levels; ++lev) {
                const Map& m = U->adj[lev];
                HIPCHK(launch_analysis_adjoint_batched(table(U, t_init), m.bmap, m.bfirst, m.nblocks, lev,
                                                       1 << (lev - 1), 1, U->mu_part[lev - 1], s));
            }
        for (int k = L - 1; k >= 0; --k) {
            const BatchImage* T = table(U, t_adj[j][k]);
            for (int lev = U->levels; lev >= 1; --lev) {
                const Map& m = U->syn[lev];
                HIPCHK(launch_synthesis_batched(T, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 0, s, 0));
            }
            HIPCHK(launch_conv_batched(T, U->conv_a.bmap, U->conv_a.bfirst, U->conv_a.nblocks, 1, U->p, nullptr, s));
            for (int pass = 0; pass < 3; ++pass)
                HIPCHK(launch_precond_batched(T, U->pre[pass].bmap, U->pre[pass].bfirst, U->pre[pass].nblocks, pass,
                                              MLBA_PRECOND_BCCB, U->nmax, s, U->any_len));
            HIPCHK(launch_conv_batched(T, U->conv_at.bmap, U->conv_at.bfirst, U->conv_at.nblocks, 0, U->p, nullptr,
                                       s));
            for (int lev = 1; lev <= U->levels; ++lev) {
                const Map& m = U->adj[lev];
                HIPCHK(launch_analysis_adjoint_batched(T, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 0,
                                                       U->mu_part[lev - 1], s));
            }
            HIPCHK(launch_psf_corr_batched(T, U->corr.bmap, U->corr.bfirst, U->corr.nblocks, U->p, first ? 1 : 0,
                                           U->corr_part, U->alpha_part, s));
            first = false;
        }
    }
    // spectral term: inverse transform of the accumulated E, then the PSF sums
    const BatchImage* T = table(U, t_end);
    HIPCHK(launch_precond_batched(T, U->pre[1].bmap, U->pre[1].bfirst, U->pre[1].nblocks, 3, MLBA_PRECOND_BCCB,
                                  U->nmax, s, U->any_len));
    HIPCHK(launch_precond_batched(T, U->pre[2].bmap, U->pre[2].bfirst, U->pre[2].nblocks, 2, MLBA_PRECOND_BCCB,
                                  U->nmax, s, U->any_len));
    HIPCHK(launch_psf_spectral_batched(T, U->count, U->p, U->spec, s));
    UnrolledSums S{};
    S.bands = U->bands;
    S.levels = U->levels;
    S.p = U->p;
    S.count = U->count;
    S.corr_blocks = U->corr.nblocks;
    for (int lev = 1; lev <= U->levels; ++lev) {
        S.mu_blocks[lev - 1] = U->adj[lev].nblocks;
        S.mu_part[lev - 1] = U->mu_part[lev - 1];
    }
    S.alpha_part = U->alpha_part;
    S.corr_part = U->corr_part;
    S.spec = U->spec;
    HIPCHK(launch_unrolled_reduce(S, dmu, dalpha, dpsf, s));
    return note_unrolled(U, s);
}

}  // extern "C"
