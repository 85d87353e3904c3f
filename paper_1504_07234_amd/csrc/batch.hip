// Batched restoration: many images of uneven sizes, each with its own PSF, alpha,
// mu and step, advanced together.  Every phase of an iteration of eq. (MLBA2)
// is one launch whose workgroups cover the tiles of all images (per-phase maps
// workgroup -> (image, tile)); each tile runs the same device body as the
// single-image path, so every image follows exactly the arithmetic of its own
// plan.  The K-iteration sequence can be captured once into a hipGraph on a
// private stream and replayed on the caller's stream; per-call data (image
// pointers, alpha, mu, delta) live in a device descriptor table that the graph
// reads at run time.
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
    int* bmap = nullptr;    // device: workgroup -> image
    int* bfirst = nullptr;  // device: image -> first workgroup
};

}  // namespace

struct mlba_batch_s {
    int count = 0, levels = 0, precond = 0, pmax = 1, nmax = 8;
    int any_len = 0;  // some image's transform takes the Bluestein form
    bool any_reflect = false;
    std::vector<mlba_plan_t> plans;
    std::vector<BatchImage> host;
    BatchImage* imgs = nullptr;
    int* maps = nullptr;  // one device buffer holding every map
    size_t maps_cap = 0;  // its size in ints: the largest over every tile choice
    Map conv_a, conv_at, fold, fill, pre[3], syn[5], ana[5], low[5], shr[5], fill_om;
    // tile choices (set by mlba_batch_autotune)
    int conv_ry[2] = {1, 1};          // output rows per thread of the A and A^T launches
    int rows_want = 0, cols_want = 0;  // transform batching caps (0: built-in choice per size)
    double* partials = nullptr;
    int* pcount = nullptr;
    double* rn = nullptr;
    int rn_cap = 0;
    hipStream_t cap = nullptr;  // private stream for graph capture
    hipGraphExec_t exec = nullptr;
    int exec_iters = -1, exec_fill = -1, exec_state = -1;
    hipEvent_t done = nullptr;  // recorded after every call that enqueues work
};

namespace {

void destroy_batch(mlba_batch_s* B) {
    if (B->done) hipEventDestroy(B->done);
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->cap) hipStreamDestroy(B->cap);
    hipFree(B->imgs);
    hipFree(B->maps);
    hipFree(B->partials);
    hipFree(B->pcount);
    hipFree(B->rn);
    delete B;
}

// Build the workgroup -> image map of one phase from per-image tile counts.
void build_map(const std::vector<int>& tiles, std::vector<int>& host_maps, std::vector<size_t>& offs, Map& m) {
    m.nblocks = 0;
    for (int t : tiles) m.nblocks += t;
    offs.push_back(host_maps.size());  // bmap offset
    for (size_t i = 0; i < tiles.size(); ++i)
        for (int t = 0; t < tiles[i]; ++t) host_maps.push_back((int)i);
    offs.push_back(host_maps.size());  // bfirst offset
    int acc = 0;
    for (int t : tiles) {
        host_maps.push_back(acc);
        acc += t;
    }
}

// Applies the batch's tile choices: per-image transform batching and residual
// partial offsets, every phase map (uploaded into the map buffer allocated at
// creation for the largest choice), descriptors and partial counts uploaded.
// Drops a captured graph (its maps are stale).  dry_run: only returns the
// map size in ints through *ints (nothing is uploaded).
int configure(mlba_batch_s* B, hipStream_t s, bool dry_run = false, size_t* ints = nullptr) {
    const int count = B->count;
    int pbase = 0;
    std::vector<int> pcount(count);
    for (int i = 0; i < count; ++i) {
        BatchImage& d = B->host[i];
        if (d.precond == MLBA_PRECOND_AR) {  // one row pair per workgroup (the transform is 2(n-1) long)
            d.fft_rows_g = d.fft_cols_c = 1;
            d.fft_rows_shift = d.fft_cols_shift = fft_seq_shift(1);
        } else if (d.precond != MLBA_PRECOND_NONE) {
            d.fft_rows_g = B->rows_want ? fft_rows_batch_at_most(d.n, B->rows_want) : fft_rows_batch(d.n);
            d.fft_cols_c = B->cols_want ? fft_cols_batch_at_most(d.n, B->cols_want) : fft_cols_batch(d.n);
            d.fft_rows_shift = fft_seq_shift(d.fft_rows_g);
            d.fft_cols_shift = fft_seq_shift(d.fft_cols_c);
        }
        d.pbase = pbase;
        pcount[i] = conv_batched_tiles(d, 1, B->conv_ry[0]);
        pbase += pcount[i];
    }
    std::vector<int> hm;
    std::vector<size_t> offs;
    std::vector<Map*> order;
    auto add = [&](Map& m, const std::vector<int>& tiles) {
        build_map(tiles, hm, offs, m);
        order.push_back(&m);
    };
    std::vector<int> t(count);
    for (int i = 0; i < count; ++i) t[i] = conv_batched_tiles(B->host[i], 1, B->conv_ry[0]);
    add(B->conv_a, t);
    for (int i = 0; i < count; ++i) t[i] = conv_batched_tiles(B->host[i], 0, B->conv_ry[1]);
    add(B->conv_at, t);
    for (int i = 0; i < count; ++i) t[i] = B->host[i].bc == MLBA_BC_REFLECT ? B->host[i].n : 0;
    add(B->fold, t);
    for (int planes : {-1, 1}) {  // the explicit state (bands planes), then the implicit one (omega)
        for (int i = 0; i < count; ++i) {
            BatchImage d = B->host[i];
            d.state_planes = planes < 0 ? d.bands : planes;
            t[i] = fill_tiles(d);
        }
        add(planes < 0 ? B->fill : B->fill_om, t);
    }
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < count; ++i) t[i] = precond_pass_tiles(B->host[i], pass);
        add(B->pre[pass], t);
    }
    for (int lev = 1; lev <= B->levels; ++lev) {
        for (int i = 0; i < count; ++i) t[i] = synthesis_level_tiles(B->host[i].N, 1 << (lev - 1));
        add(B->syn[lev], t);
        for (int i = 0; i < count; ++i) t[i] = analysis_level_tiles(B->host[i].N, 1 << (lev - 1));
        add(B->ana[lev], t);
        for (int i = 0; i < count; ++i) t[i] = lev < B->levels ? lowpass_level_tiles(B->host[i].N) : 0;
        add(B->low[lev], t);
        for (int i = 0; i < count; ++i) t[i] = shrink_level_tiles(B->host[i].N, 1 << (lev - 1));
        add(B->shr[lev], t);
    }
    if (dry_run) {
        *ints = hm.size();
        return MLBA_OK;
    }
    if (hm.size() > B->maps_cap) return MLBA_EINVAL;  // cannot happen: sized for the largest choice
    if (B->exec) {
        HIPCHK(hipGraphExecDestroy(B->exec));
        B->exec = nullptr;
    }
    for (size_t q = 0; q < order.size(); ++q) {
        order[q]->bmap = B->maps + offs[2 * q];
        order[q]->bfirst = B->maps + offs[2 * q + 1];
    }
    HIPCHK(hipMemcpyAsync(B->maps, hm.data(), hm.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B->pcount, pcount.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B->imgs, B->host.data(), count * sizeof(BatchImage), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return MLBA_OK;
}

// u (f when final_out) = W^T(delta S_mu(W omega)) of every image: the low-pass
// chain, then the shrink-synthesis levels from the top
int enqueue_shrink_synthesis(mlba_batch_s* B, int final_out, hipStream_t s) {
    const BatchImage* I = B->imgs;
    for (int lev = 1; lev < B->levels; ++lev) {
        const Map& m = B->low[lev];
        HIPCHK(launch_lowpass_batched(I, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), s));
    }
    for (int lev = B->levels; lev >= 1; --lev) {
        const Map& m = B->shr[lev];
        HIPCHK(launch_shrink_synthesis_batched(I, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1),
                                               lev == B->levels ? 1 : 0, final_out, s));
    }
    return MLBA_OK;
}

// Implicit state: per iteration the shrink-synthesis, r = g - A u, t = P r and
// omega += A^T t (accumulated by the A^T launch, or by the fold of the
// reflective model); no analysis.
int enqueue_implicit(mlba_batch_s* B, int iters, bool fill_state, hipStream_t s) {
    const BatchImage* I = B->imgs;
    if (fill_state) HIPCHK(launch_fill_batched(I, B->fill_om.bmap, B->fill_om.bfirst, B->fill_om.nblocks, s));
    for (int k = 0; k < iters; ++k) {
        STCHK(enqueue_shrink_synthesis(B, 0, s));
        HIPCHK(launch_conv_batched(I, B->conv_a.bmap, B->conv_a.bfirst, B->conv_a.nblocks, 1, B->pmax, B->partials,
                                   s, B->conv_ry[0]));
        HIPCHK(launch_sum_partials_batched(I, B->partials, B->pcount, B->count, k, s));
        if (B->precond != MLBA_PRECOND_NONE)
            for (int pass = 0; pass < 3; ++pass)
                HIPCHK(launch_precond_batched(I, B->pre[pass].bmap, B->pre[pass].bfirst, B->pre[pass].nblocks, pass,
                                              B->precond, B->nmax, s, B->any_len));
        HIPCHK(launch_conv_batched(I, B->conv_at.bmap, B->conv_at.bfirst, B->conv_at.nblocks, 0, B->pmax, nullptr,
                                   s, B->conv_ry[1]));
        if (B->any_reflect) HIPCHK(launch_fold_batched(I, B->fold.bmap, B->fold.bfirst, B->fold.nblocks, s));
    }
    return enqueue_shrink_synthesis(B, 1, s);
}

int enqueue(mlba_batch_s* B, int iters, bool fill_state, bool implicit, hipStream_t s) {
    if (implicit) return enqueue_implicit(B, iters, fill_state, s);
    const BatchImage* I = B->imgs;
    if (fill_state) HIPCHK(launch_fill_batched(I, B->fill.bmap, B->fill.bfirst, B->fill.nblocks, s));
    for (int k = 0; k < iters; ++k) {
        for (int lev = B->levels; lev >= 1; --lev) {
            const Map& m = B->syn[lev];
            HIPCHK(launch_synthesis_batched(I, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 0, s));
        }
        HIPCHK(launch_conv_batched(I, B->conv_a.bmap, B->conv_a.bfirst, B->conv_a.nblocks, 1, B->pmax, B->partials,
                                   s, B->conv_ry[0]));
        HIPCHK(launch_sum_partials_batched(I, B->partials, B->pcount, B->count, k, s));
        if (B->precond != MLBA_PRECOND_NONE)
            for (int pass = 0; pass < 3; ++pass)
                HIPCHK(launch_precond_batched(I, B->pre[pass].bmap, B->pre[pass].bfirst, B->pre[pass].nblocks, pass,
                                              B->precond, B->nmax, s, B->any_len));
        HIPCHK(launch_conv_batched(I, B->conv_at.bmap, B->conv_at.bfirst, B->conv_at.nblocks, 0, B->pmax, nullptr,
                                   s, B->conv_ry[1]));
        if (B->any_reflect) HIPCHK(launch_fold_batched(I, B->fold.bmap, B->fold.bfirst, B->fold.nblocks, s));
        for (int lev = 1; lev <= B->levels; ++lev) {
            const Map& m = B->ana[lev];
            HIPCHK(launch_analysis_batched(I, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), s));
        }
    }
    for (int lev = B->levels; lev >= 1; --lev) {
        const Map& m = B->syn[lev];
        HIPCHK(launch_synthesis_batched(I, m.bmap, m.bfirst, m.nblocks, lev, 1 << (lev - 1), 1, s));
    }
    return MLBA_OK;
}

}  // namespace

namespace {

// Mean milliseconds of `reps` launches of `phase` after one untimed launch.
template <class F>
int time_phase(F phase, int reps, hipStream_t s, double* ms) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        mlba_internal_set_hip(err);
        return MLBA_EHIP;
    }
    int st = phase();
    if (st >= 0) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st >= 0; ++r) st = phase();
        (void)hipEventRecord(e1, s);
        err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) {
            mlba_internal_set_hip(err);
            st = MLBA_EHIP;
        }
        *ms = (double)t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" {

int mlba_batch_create(mlba_batch_t* batch, int count, const mlba_plan_t* plans, int max_iters, hipStream_t s) {
    if (!batch || !plans || count < 1 || max_iters < 1) return MLBA_EINVAL;
    *batch = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return MLBA_EINVAL;
        if (plans[i]->levels != plans[0]->levels || plans[i]->precond != plans[0]->precond) return MLBA_EINVAL;
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return MLBA_EINVAL;  // one image per plan (the plan holds its buffers)
    }
    mlba_batch_s* B = new (std::nothrow) mlba_batch_s();
    if (!B) return MLBA_ENOMEM;
    B->count = count;
    B->levels = plans[0]->levels;
    B->precond = plans[0]->precond;
    B->plans.assign(plans, plans + count);
    B->rn_cap = max_iters;
    B->host.resize(count);
    int pmax_parts = 0;  // residual partials with one row per thread (the most tiles)
    for (int i = 0; i < count; ++i) {
        B->host[i] = plan_desc(plans[i]);
        B->pmax = std::max(B->pmax, plans[i]->p);
        B->nmax = std::max(B->nmax, plans[i]->n);
        if (plans[i]->fd.m > 0) B->any_len = 1;  // a Bluestein-form transform
        B->any_reflect = B->any_reflect || plans[i]->bc == MLBA_BC_REFLECT;
        pmax_parts += conv_batched_tiles(B->host[i], 1, 1);
    }
    hipError_t e = hipMalloc(&B->imgs, count * sizeof(BatchImage));
    if (e == hipSuccess) e = hipMalloc(&B->partials, (size_t)std::max(pmax_parts, 1) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&B->pcount, count * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&B->rn, (size_t)count * max_iters * sizeof(double));
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        destroy_batch(B);
        return MLBA_ENOMEM;
    }
    for (int i = 0; i < count; ++i) B->host[i].rn = B->rn + (size_t)i * max_iters;
    // the map buffer for the tile choice with the most workgroups in every
    // phase (one output row per thread, one row pair and one column per
    // transform workgroup), so that changing the choice allocates nothing
    B->conv_ry[0] = B->conv_ry[1] = 1;
    B->rows_want = B->cols_want = 1;
    size_t need = 0, need0 = 0;
    int st = configure(B, s, true, &need);
    B->rows_want = B->cols_want = 0;
    if (st >= 0) st = configure(B, s, true, &need0);
    if (st < 0) {
        destroy_batch(B);
        return st;
    }
    B->maps_cap = std::max(need, need0);
    e = hipMalloc(&B->maps, B->maps_cap * sizeof(int));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        destroy_batch(B);
        return MLBA_ENOMEM;
    }
    st = configure(B, s);
    if (st < 0) {
        destroy_batch(B);
        return st;
    }
    e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        destroy_batch(B);
        return MLBA_EHIP;
    }
    *batch = B;
    return MLBA_OK;
}

int mlba_batch_autotune(mlba_batch_t B, int reps, mlba_batch_tuning* out, hipStream_t s) {
    if (!B || reps < 1) return MLBA_EINVAL;
    const BatchImage* I = B->imgs;
    // A and A^T: one or two output rows per thread
    for (int which = 0; which < 2; ++which) {
        double best = 1e300;
        int best_ry = 1;
        for (int ry = 1; ry <= 2; ++ry) {
            B->conv_ry[which] = ry;
            STCHK(configure(B, s));
            const Map& m = which == 0 ? B->conv_a : B->conv_at;
            double ms = 0.0;
            STCHK(time_phase([&]() -> int {
                HIPCHK(launch_conv_batched(I, m.bmap, m.bfirst, m.nblocks, which == 0 ? 1 : 0, B->pmax, nullptr, s,
                                           ry));
                return MLBA_OK;
            }, reps, s, &ms));
            if (out) out->conv_ms[which][ry - 1] = ms;
            if (ms < best) {
                best = ms;
                best_ry = ry;
            }
        }
        B->conv_ry[which] = best_ry;
    }
    if (B->precond != MLBA_PRECOND_NONE) {
        // row passes (forward and inverse): caps on the row pairs per workgroup
        static const int rows_cand[MLBA_TUNE_ROWS] = {0, 1, 2, 4};
        double best = 1e300;
        int best_w = 0;
        for (int c = 0; c < MLBA_TUNE_ROWS; ++c) {
            B->rows_want = rows_cand[c];
            STCHK(configure(B, s));
            double ms = 0.0;
            STCHK(time_phase([&]() -> int {
                for (int pass = 0; pass < 3; pass += 2)
                    HIPCHK(launch_precond_batched(I, B->pre[pass].bmap, B->pre[pass].bfirst, B->pre[pass].nblocks,
                                                  pass, B->precond, B->nmax, s, B->any_len));
                return MLBA_OK;
            }, reps, s, &ms));
            if (out) out->rows_ms[c] = ms;
            if (ms < best) {
                best = ms;
                best_w = rows_cand[c];
            }
        }
        B->rows_want = best_w;
        // column pass: caps on the columns per workgroup
        static const int cols_cand[MLBA_TUNE_COLS] = {0, 1, 2, 4, 8, 16};
        best = 1e300;
        best_w = 0;
        for (int c = 0; c < MLBA_TUNE_COLS; ++c) {
            B->cols_want = cols_cand[c];
            STCHK(configure(B, s));
            double ms = 0.0;
            STCHK(time_phase([&]() -> int {
                HIPCHK(launch_precond_batched(I, B->pre[1].bmap, B->pre[1].bfirst, B->pre[1].nblocks, 1, B->precond,
                                              B->nmax, s, B->any_len));
                return MLBA_OK;
            }, reps, s, &ms));
            if (out) out->cols_ms[c] = ms;
            if (ms < best) {
                best = ms;
                best_w = cols_cand[c];
            }
        }
        B->cols_want = best_w;
    }
    STCHK(configure(B, s));
    if (out) {
        out->conv_rows[0] = B->conv_ry[0];
        out->conv_rows[1] = B->conv_ry[1];
        out->fft_rows_cap = B->rows_want;
        out->fft_cols_cap = B->cols_want;
    }
    return MLBA_OK;
}

int mlba_batch_set_tiles(mlba_batch_t B, const mlba_batch_tuning* choice, hipStream_t s) {
    if (!B || !choice) return MLBA_EINVAL;
    for (int w = 0; w < 2; ++w)
        if (choice->conv_rows[w] != 1 && choice->conv_rows[w] != 2) return MLBA_EINVAL;
    if (choice->fft_rows_cap < 0 || choice->fft_cols_cap < 0) return MLBA_EINVAL;
    B->conv_ry[0] = choice->conv_rows[0];
    B->conv_ry[1] = choice->conv_rows[1];
    B->rows_want = choice->fft_rows_cap;
    B->cols_want = choice->fft_cols_cap;
    return configure(B, s);
}

int mlba_batch_destroy(mlba_batch_t B) {
    if (!B) return MLBA_EINVAL;
    if (B->done) (void)hipEventSynchronize(B->done);  // the batch's last enqueued work
    destroy_batch(B);
    return MLBA_OK;
}

int mlba_batch_restore(mlba_batch_t B, const float* const* g, const double* alpha, const double* mu, int n_mu,
                       const double* delta, int iters, float* const* f_out, float* const* z_state, double* rnorm_out,
                       int state, int use_graph, hipStream_t s) {
    if (!B || !g || !alpha || !mu || !delta || !f_out || iters < 0 || iters > B->rn_cap) return MLBA_EINVAL;
    if (state != MLBA_STATE_EXPLICIT && state != MLBA_STATE_IMPLICIT) return MLBA_EINVAL;
    const bool implicit = state == MLBA_STATE_IMPLICIT;
    const int count = B->count;
    const int bands = 8 * B->levels + 1;
    if (n_mu != 1 && n_mu != bands) return MLBA_EINVAL;
    for (int i = 0; i < count; ++i) {
        BatchImage& d = B->host[i];
        if (!g[i] || !f_out[i]) return MLBA_EINVAL;
        if (B->precond != MLBA_PRECOND_NONE && !(alpha[i] > 0.0)) return MLBA_EINVAL;
        double dl = delta[i];
        if (!(dl > 0.0)) STCHK(mlba_internal_auto_delta(B->plans[i], alpha[i], &dl, s));
        d.alpha = (float)alpha[i];
        d.delta = (float)dl;
        for (int b = 0; b < bands; ++b) {
            const double m = mu[(size_t)i * n_mu + (n_mu == 1 ? 0 : b)];
            if (!(m >= 0.0) || !isfinite(m)) return MLBA_EINVAL;
            d.mu[b] = (float)m;
        }
        d.g = g[i];
        d.f = f_out[i];
        if (implicit) {
            d.z = z_state ? z_state[i] : B->plans[i]->omega;
            d.w = d.z;  // omega += A^T t
            d.blur_acc = 1;
            d.state_planes = 1;
            for (int lev = 1; lev <= B->levels; ++lev) {
                LevelMu lm;
                lm.low = d.mu[0];
                for (int q = 0; q < 8; ++q) lm.band[q] = d.mu[1 + 8 * (lev - 1) + q];
                d.ss[lev - 1] = ss_coef(lm, d.delta, lev < B->levels);
            }
        } else {
            d.z = z_state ? z_state[i] : B->plans[i]->z;
            d.w = B->plans[i]->w;
            d.blur_acc = 0;
            d.state_planes = d.bands;
        }
        d.zin = d.z;
        if (!d.z) return MLBA_EINVAL;
    }
    HIPCHK(hipMemcpyAsync(B->imgs, B->host.data(), count * sizeof(BatchImage), hipMemcpyHostToDevice, s));
    const bool fill_state = z_state == nullptr;
    if (use_graph) {
        if (!B->exec || B->exec_iters != iters || B->exec_fill != (int)fill_state || B->exec_state != state) {
            if (B->exec) {
                HIPCHK(hipGraphExecDestroy(B->exec));
                B->exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
            const int st = enqueue(B, iters, fill_state, implicit, B->cap);
            hipError_t e = hipStreamEndCapture(B->cap, &graph);
            if (st < 0) {
                if (graph) hipGraphDestroy(graph);
                return st;
            }
            HIPCHK(e);
            e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            HIPCHK(e);
            B->exec_iters = iters;
            B->exec_fill = (int)fill_state;
            B->exec_state = state;
        }
        HIPCHK(hipGraphLaunch(B->exec, s));
    } else {
        STCHK(enqueue(B, iters, fill_state, implicit, s));
    }
    // the batch's and its plans' completion events (their buffers were used)
    HIPCHK(hipEventRecord(B->done, s));
    for (mlba_plan_t P : B->plans)
        if (P->done) HIPCHK(hipEventRecord(P->done, s));
    if (rnorm_out && iters > 0) {
        std::vector<double> buf((size_t)count * B->rn_cap);
        HIPCHK(hipMemcpyAsync(buf.data(), B->rn, buf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int status = MLBA_OK;
        for (int i = 0; i < count; ++i) {
            const double first = sqrt(buf[(size_t)i * B->rn_cap]);
            for (int k = 0; k < iters; ++k) {
                const double v = sqrt(buf[(size_t)i * B->rn_cap + k]);
                rnorm_out[(size_t)i * iters + k] = v;
                if (!isfinite(v) || v > 1e3 * first) status = MLBA_WARN_DIVERGED;
            }
        }
        return status;
    }
    return MLBA_OK;
}

}  // extern "C"
