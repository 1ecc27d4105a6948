// C ABI of libpmf (include/pmf.h): validation, device state, host orchestration
// of the generic kernels, state images.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.h"
#include "kernels.h"

namespace pmf {

thread_local std::string g_last_error;

pmf_status fail(pmf_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

pmf_status hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PMF_E_DEVICE;
}

void* ctx_alloc(pmf_ctx* ctx, size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 16;
    if (ctx->has_alloc) return ctx->alloc.alloc(bytes, ctx->alloc.user, st);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void ctx_free(pmf_ctx* ctx, void* p, hipStream_t st) {
    if (!p) return;
    if (ctx->has_alloc) ctx->alloc.free(p, ctx->alloc.user, st);
    else (void)hipFree(p);
}

// ---------------------------------------------------------------- host math

static bool chol_ok(const double* S, int n) {
    double L[MSQ] = {0};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = S[i * MS + j];
            for (int k = 0; k < j; ++k) s -= L[i * MS + k] * L[j * MS + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * MS + i] = std::sqrt(s);
            } else {
                L[i * MS + j] = s / L[j * MS + j];
            }
        }
    return true;
}

static void diffusion(const pmf_model& m, double* D) {
    mat_zero(D);
    const int n = m.nx;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += m.Q[i * n + k] * m.Q[j * n + k];
            D[i * MS + j] = s;
        }
}

static void load_square(const double* src, int n, double* dst) {
    mat_zero(dst);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) dst[i * MS + j] = src[i * n + j];
}

// Chebyshev-Gauss-Lobatto nodes v_k = -cos(k pi / n), n = N+1, ascending.
static std::vector<double> cgl(int N) {
    const int n = N + 1;
    std::vector<double> v(n + 1);
    for (int k = 0; k <= n; ++k) v[k] = -std::cos(k * M_PI / n);
    return v;
}

// Interior first/second differentiation matrices (row-major N x N) of the
// polynomial interpolant through the N+2 CGL nodes with zero end values.
void cheb_matrices(int N, std::vector<double>& D1, std::vector<double>& D2) {
    const std::vector<double> v = cgl(N);
    const int n1 = N + 2;
    std::vector<double> D((size_t)n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i) {
        double rs = 0.0;
        for (int j = 0; j < n1; ++j) {
            if (i == j) continue;
            const double ci = (i == 0 || i == n1 - 1) ? 2.0 : 1.0;
            const double cj = (j == 0 || j == n1 - 1) ? 2.0 : 1.0;
            const double sgn = ((i + j) % 2) ? -1.0 : 1.0;
            const double val = (ci / cj) * sgn / (v[i] - v[j]);
            D[(size_t)i * n1 + j] = val;
            rs += val;
        }
        D[(size_t)i * n1 + i] = -rs;
    }
    D1.assign((size_t)N * N, 0.0);
    D2.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            D1[(size_t)i * N + j] = D[(size_t)(i + 1) * n1 + (j + 1)];
            double s = 0.0;
            for (int k = 0; k < n1; ++k) s += D[(size_t)(i + 1) * n1 + k] * D[(size_t)k * n1 + (j + 1)];
            D2[(size_t)i * N + j] = s;
        }
}

// Clenshaw-Curtis weights of the N+2 CGL nodes (closed form).
static std::vector<double> clenshaw_curtis(int N) {
    const int n = N + 1;
    std::vector<double> w(n + 1, 0.0);
    std::vector<double> vv(n - 1, 1.0);
    if (n % 2 == 0) {
        w[0] = w[n] = 1.0 / ((double)n * n - 1.0);
        for (int k = 1; k <= n / 2 - 1; ++k)
            for (int i = 1; i < n; ++i) vv[i - 1] -= 2.0 * std::cos(2.0 * k * i * M_PI / n) / (4.0 * k * k - 1.0);
        for (int i = 1; i < n; ++i) vv[i - 1] -= std::cos(n * i * M_PI / n) / ((double)n * n - 1.0);
    } else {
        w[0] = w[n] = 1.0 / ((double)n * n);
        for (int k = 1; k <= (n - 1) / 2; ++k)
            for (int i = 1; i < n; ++i) vv[i - 1] -= 2.0 * std::cos(2.0 * k * i * M_PI / n) / (4.0 * k * k - 1.0);
    }
    for (int i = 1; i < n; ++i) w[i] = 2.0 * vv[i - 1] / n;
    return w;
}

static double rho_axis(int grid, int N) {
    if (grid == PMF_GRID_FOURIER) return M_PI;
    std::vector<double> D1, D2;
    cheb_matrices(N, D1, D2);
    double best = 0.0;
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += std::fabs(D2[(size_t)i * N + j]);
        best = std::max(best, s);
    }
    return std::sqrt(best);
}

static bool design_grid_host(const pmf_model& m, const double* Wnom, const double* mean, const double* cov,
                             Grid& g) {
    mat_zero(g.M);
    for (int a = 0; a < m.nx; ++a) {
        const double v = cov[a * MS + a] + Wnom[a * MS + a];
        if (!(v > 0.0) || !std::isfinite(v)) return false;
        const double h = m.span_sigmas * std::sqrt(v);
        g.M[a * MS + a] = (m.grid == PMF_GRID_FOURIER) ? 2.0 * h / m.N[a] : h;
        g.c[a] = mean[a];
    }
    for (int a = m.nx; a < MS; ++a) g.c[a] = 0.0;
    grid_finish(g, m.nx);
    return true;
}

// ---------------------------------------------------------------- validation

static pmf_status validate_model(const pmf_model* m) {
    if (!m) return fail(PMF_E_INVALID, "model is NULL");
    if (m->nx < 1 || m->nx > MAXNX) return fail(PMF_E_INVALID, "nx must be 1..4");
    if (m->grid != PMF_GRID_FOURIER && m->grid != PMF_GRID_CHEBYSHEV)
        return fail(PMF_E_INVALID, "unknown grid kind");
    if (m->grid == PMF_GRID_CHEBYSHEV && m->nx > 3) return fail(PMF_E_INVALID, "Chebyshev grids: nx must be 1..3");
    long ntot = 1;
    for (int a = 0; a < m->nx; ++a) {
        const int n = m->N[a];
        if (n < 4 || n > 256) return fail(PMF_E_INVALID, "N per axis must be 4..256");
        if (m->grid == PMF_GRID_FOURIER && (n % 2 != 0 || make_plan(n).np < 0))
            return fail(PMF_E_INVALID, "Fourier N must be even and of the form 2^a 3^b 5^c 7^d 11^e 13^f 17^g");
        if ((m->integrator == PMF_INT_FDM || m->integrator == PMF_INT_SINE) && make_plan(2 * (n + 1)).np < 0)
            return fail(PMF_E_INVALID, "the sine transform needs 2 (N + 1) of the form 2^a 3^b 5^c 7^d 11^e 13^f 17^g");
        ntot *= n;
    }
    if (ntot > (1L << 24)) return fail(PMF_E_INVALID, "grid larger than 2^24 points");
    if (m->integrator < 0 || m->integrator > 4) return fail(PMF_E_INVALID, "unknown integrator");
    if (m->integrator == PMF_INT_FDM || m->integrator == PMF_INT_SINE) {
        if (m->grid != PMF_GRID_FOURIER)
            return fail(PMF_E_INVALID, "the finite-difference and sine-series forms need a Fourier grid");
        double Dm[MSQ];
        diffusion(*m, Dm);
        for (int i = 0; i < m->nx; ++i)
            for (int j = 0; j < m->nx; ++j)
                if (i != j && (m->A[i * m->nx + j] != 0.0 || Dm[i * MS + j] != 0.0))
                    return fail(PMF_E_INVALID, "the finite-difference and sine-series forms need diagonal A and D");
    }
    if (m->grid == PMF_GRID_CHEBYSHEV && m->integrator != PMF_INT_RK4)
        return fail(PMF_E_INVALID, "Chebyshev grids support the RK4 integrator only");
    if (m->substeps < 1 || m->substeps > LMAX) return fail(PMF_E_INVALID, "substeps must be 1..4096");
    if (m->precision != PMF_FP64 && m->precision != PMF_FP32) return fail(PMF_E_INVALID, "unknown precision");
    if (m->interp != PMF_INTERP_AUTO && m->interp != PMF_INTERP_LAGRANGE)
        return fail(PMF_E_INVALID, "unknown interpolation mode");
    if (!(m->span_sigmas > 0.0) || !std::isfinite(m->span_sigmas)) return fail(PMF_E_INVALID, "span_sigmas <= 0");
    if (!(m->t_nominal > 0.0) || !std::isfinite(m->t_nominal)) return fail(PMF_E_INVALID, "t_nominal <= 0");
    for (int i = 0; i < m->nx * m->nx; ++i)
        if (!std::isfinite(m->A[i]) || !std::isfinite(m->Q[i])) return fail(PMF_E_INVALID, "non-finite A or Q");
    if (m->meas_kind < 0 || m->meas_kind > 3) return fail(PMF_E_INVALID, "unknown measurement kind");
    if (m->meas_kind == PMF_H_LINEAR) {
        if (m->nz < 1 || m->nz > 3) return fail(PMF_E_INVALID, "nz must be 1..3");
    } else if (m->nz != 1) {
        return fail(PMF_E_INVALID, "nonlinear measurements have nz = 1");
    }
    if (m->meas_kind == PMF_H_TERRAIN) {
        if (m->nterrain < 1 || m->nterrain > PMF_MAX_TERRAIN)
            return fail(PMF_E_INVALID, "nterrain must be 1..8");
        for (int i = 0; i < 6 * m->nterrain; ++i)
            if (!std::isfinite(m->terrain[i])) return fail(PMF_E_INVALID, "non-finite terrain parameter");
    }
    if (m->noise_ncomp < 1 || m->noise_ncomp > MAXMIX) return fail(PMF_E_INVALID, "noise_ncomp must be 1..4");
    for (int g = 0; g < m->noise_ncomp; ++g) {
        if (!(m->noise_w[g] > 0.0)) return fail(PMF_E_INVALID, "noise weights must be > 0");
        double R[MSQ];
        load_square(m->noise_cov + 9 * g, m->nz, R);
        if (!chol_ok(R, m->nz)) return fail(PMF_E_INVALID, "noise covariance not positive definite");
    }
    return PMF_OK;
}

pmf_status check_model(const pmf_model* m) { return validate_model(m); }

static pmf_status validate_prior(const pmf_prior* p, int nx) {
    if (!p) return fail(PMF_E_INVALID, "prior is NULL");
    if (p->ncomp < 1 || p->ncomp > MAXMIX) return fail(PMF_E_INVALID, "prior ncomp must be 1..4");
    for (int g = 0; g < p->ncomp; ++g) {
        if (!(p->w[g] > 0.0)) return fail(PMF_E_INVALID, "prior weights must be > 0");
        double C[MSQ];
        load_square(p->cov + MSQ * g, nx, C);
        if (!chol_ok(C, nx)) return fail(PMF_E_INVALID, "prior covariance not positive definite");
    }
    return PMF_OK;
}

static void build_kmodel(const pmf_model& m, KModel& k, double* Wnom) {
    std::memset(&k, 0, sizeof(k));
    k.nx = m.nx;
    k.grid = m.grid;
    k.meas = m.meas_kind;
    k.nz = m.nz;
    k.ncomp = m.noise_ncomp;
    k.interp = m.interp;
    k.integ = m.integrator;
    k.prec = m.precision;
    k.ntot = 1;
    for (int a = 0; a < MS; ++a) {
        k.N[a] = a < m.nx ? m.N[a] : 1;
        k.ntot *= k.N[a];
    }
    for (int i = 0; i < m.nz; ++i)
        for (int j = 0; j < m.nx; ++j) k.H[i * MS + j] = m.H[i * m.nx + j];
    for (int i = 0; i < 4; ++i) k.hp[i] = m.hparam[i];
    if (m.meas_kind == PMF_H_TERRAIN) {
        k.nterr = m.nterrain;
        for (int c = 0; c < m.nterrain; ++c) {
            k.terr[c][0] = m.terrain[6 * c];
            k.terr[c][1] = m.terrain[6 * c + 1];
            for (int a = 0; a < m.nx; ++a) k.terr[c][2 + a] = m.terrain[6 * c + 2 + a];
        }
    }
    double wsum = 0.0;
    for (int g = 0; g < m.noise_ncomp; ++g) wsum += m.noise_w[g];
    for (int g = 0; g < m.noise_ncomp; ++g) {
        double R[MSQ], Ri[MSQ];
        load_square(m.noise_cov + 9 * g, m.nz, R);
        const double det = mat_inv(Ri, R, m.nz);
        mat_copy(k.nRi[g], Ri);
        k.lw[g] = std::log(m.noise_w[g] / wsum) - 0.5 * (m.nz * std::log(2.0 * M_PI) + std::log(det));
        for (int i = 0; i < m.nz; ++i) k.nmean[g][i] = m.noise_mean[3 * g + i];
    }
    int maxn = 1;
    for (int a = 0; a < m.nx; ++a) maxn = m.N[a] > maxn ? m.N[a] : maxn;
    k.wstride = maxn * maxn;
    k.span = m.span_sigmas;
    double A[MSQ], D[MSQ];
    load_square(m.A, m.nx, A);
    diffusion(m, D);
    w_integral(Wnom, A, D, m.t_nominal, m.nx);
    mat_copy(k.Wnom, Wnom);
    for (int a = 0; a < m.nx; ++a) k.rho[a] = rho_axis(m.grid, m.N[a]);
}

static void fill_tables(const pmf_model& m, std::vector<double>& tab) {
    tab.assign((size_t)MS * TAB_STRIDE, 0.0);
    for (int a = 0; a < m.nx; ++a) {
        double* t = tab.data() + (size_t)a * TAB_STRIDE;
        const int n = m.N[a];
        if (m.grid == PMF_GRID_FOURIER) {
            for (int j = 0; j < n; ++j) {
                t[j] = (double)(j - n / 2);
                t[TAB_QW + j] = 1.0;
            }
        } else {
            const std::vector<double> v = cgl(n);
            const std::vector<double> w = clenshaw_curtis(n);
            for (int j = 0; j < n; ++j) {
                t[j] = v[j + 1];
                t[TAB_QW + j] = w[j + 1];
            }
            for (int k = 0; k < n + 2; ++k) {
                t[TAB_V + k] = v[k];
                const double delta = (k == 0 || k == n + 1) ? 0.5 : 1.0;
                t[TAB_BETA + k] = ((k % 2) ? -1.0 : 1.0) * delta;
            }
        }
    }
}


// Device bytes pmf_create allocates for a (validated) model, in the same order and
// sizes; the server admits tracks by it before creating them.
size_t filter_device_bytes(const pmf_model& model) {
    KModel km{};
    double Wn[MSQ];
    build_kmodel(model, km, Wn);
    const size_t es = model.precision == PMF_FP64 ? sizeof(double) : sizeof(float);
    const size_t ntot = (size_t)km.ntot;
    int chunk, nb;
    red_partition(km.ntot, &chunk, &nb);
    size_t b = 4 * ntot * es;
    if (model.grid == PMF_GRID_FOURIER) b += ntot * es * 2;
    b += (size_t)nb * NPART * sizeof(double) + (size_t)nb * sizeof(double);
    b += (size_t)(2 * LMAX + 1) * PACK * sizeof(double);
    b += (size_t)model.nx * km.wstride * sizeof(double);
    b += (size_t)MS * TAB_STRIDE * sizeof(double);
    b += sizeof(DevDesc);
    if (model.grid == PMF_GRID_CHEBYSHEV) b += 2 * (size_t)3 * 256 * 256 * es + 5 * ntot * es;
    return b;
}

}  // namespace pmf

using namespace pmf;

// ================================================================ C ABI

extern "C" {

pmf_status pmf_model_check(const pmf_model* model, int* fusable, char* why, size_t why_len) {
    using namespace pmf;
    if (why && why_len) why[0] = '\0';
    const pmf_status s = check_model(model);
    if (s != PMF_OK) return s;
    if (fusable) {
        std::string reason;
        const bool ok = model_fusable(*model, &reason);
        *fusable = ok ? 1 : 0;
        if (!ok && why && why_len) {
            const size_t k = std::min(why_len - 1, reason.size());
            std::memcpy(why, reason.data(), k);
            why[k] = '\0';
        }
    }
    return PMF_OK;
}

const char* pmf_last_error(void) { return g_last_error.c_str(); }

pmf_status pmf_ctx_create(int device, const pmf_allocator* a, pmf_ctx** out) {
    if (!out) return fail(PMF_E_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(PMF_E_INVALID, "no such device");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (a && (!a->alloc || !a->free)) return fail(PMF_E_INVALID, "allocator needs alloc and free");
    pmf_ctx* c = new pmf_ctx();
    c->device = device;
    c->has_alloc = a != nullptr;
    if (a) c->alloc = *a;
    *out = c;
    return PMF_OK;
}

void pmf_ctx_destroy(pmf_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    batch_cache_release(ctx);
    for (hipEvent_t ev : ctx->ev_pool) (void)hipEventDestroy(ev);
    delete ctx;
}


pmf_status pmf_create(pmf_ctx* ctx, const pmf_model* model, const pmf_prior* prior, pmf_filter** out) {
    if (!ctx || !out) return fail(PMF_E_INVALID, "ctx/out is NULL");
    *out = nullptr;
    pmf_status s = validate_model(model);
    if (s != PMF_OK) return s;
    s = validate_prior(prior, model->nx);
    if (s != PMF_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

    pmf_filter* f = new pmf_filter();
    f->ctx = ctx;
    f->model = *model;
    build_kmodel(*model, f->km, f->Wnom);
    f->ntot = f->km.ntot;
    f->es = model->precision == PMF_FP64 ? sizeof(double) : sizeof(float);
    red_partition(f->ntot, &f->chunk, &f->nb);
    const hipStream_t st = nullptr;
    bool okalloc = true;
    auto A = [&](size_t bytes) {
        void* p = ctx_alloc(ctx, bytes, st);
        if (!p) okalloc = false;
        f->bytes += bytes;
        return p;
    };
    for (int i = 0; i < 4; ++i) f->buf[i] = A(f->ntot * f->es);
    if (model->grid == PMF_GRID_FOURIER) f->cbuf = A(f->ntot * f->es * 2);
    f->part = static_cast<double*>(A((size_t)f->nb * NPART * sizeof(double)));
    f->bfac = static_cast<double*>(A((size_t)f->nb * sizeof(double)));
    f->coef = static_cast<double*>(A((size_t)(2 * LMAX + 1) * PACK * sizeof(double)));
    f->W = static_cast<double*>(A((size_t)model->nx * f->km.wstride * sizeof(double)));
    f->tab = static_cast<double*>(A((size_t)MS * TAB_STRIDE * sizeof(double)));
    f->desc = static_cast<DevDesc*>(A(sizeof(DevDesc)));
    if (model->grid == PMF_GRID_CHEBYSHEV) {
        f->D1 = A((size_t)3 * 256 * 256 * f->es);
        f->D2 = A((size_t)3 * 256 * 256 * f->es);
        for (int i = 0; i < 5; ++i) f->rk[i] = A(f->ntot * f->es);
    }
    {
        std::string why;
        if (batch_fusable(f, &why)) {
            f->dconst = A(fused_const_bytes());
            f->dconst_T = -1.0;
        }
    }
    if (!okalloc) {
        pmf_destroy(f);
        return fail(PMF_E_NOMEM, "device allocation failed");
    }
    if (f->bytes != filter_device_bytes(*model) + (f->dconst ? fused_const_bytes() : 0)) {
        pmf_destroy(f);
        return fail(PMF_E_DEVICE, "device footprint differs from filter_device_bytes (library error)");
    }
    f->cur = 0;

    // axis tables and (Chebyshev) differentiation matrices
    std::vector<double> tab;
    fill_tables(*model, tab);
    e = hipMemcpy(f->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pmf_destroy(f);
        return hip_fail(e, "upload tables");
    }
    if (model->grid == PMF_GRID_CHEBYSHEV) {
        std::vector<double> d1all((size_t)3 * 256 * 256, 0.0), d2all((size_t)3 * 256 * 256, 0.0);
        for (int a = 0; a < model->nx; ++a) {
            std::vector<double> D1, D2;
            cheb_matrices(model->N[a], D1, D2);
            std::copy(D1.begin(), D1.end(), d1all.begin() + (size_t)a * 256 * 256);
            std::copy(D2.begin(), D2.end(), d2all.begin() + (size_t)a * 256 * 256);
        }
        if (f->es == sizeof(double)) {
            e = hipMemcpy(f->D1, d1all.data(), d1all.size() * 8, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(f->D2, d2all.data(), d2all.size() * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> a1(d1all.begin(), d1all.end()), a2(d2all.begin(), d2all.end());
            e = hipMemcpy(f->D1, a1.data(), a1.size() * 4, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(f->D2, a2.data(), a2.size() * 4, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            pmf_destroy(f);
            return hip_fail(e, "upload differentiation matrices");
        }
        f->cheb_d32_ready = false;
    }

    // prior moments -> first grid
    const int nx = model->nx;
    double wsum = 0.0, mean[MS] = {0, 0, 0, 0}, cov[MSQ];
    mat_zero(cov);
    for (int g = 0; g < prior->ncomp; ++g) wsum += prior->w[g];
    for (int g = 0; g < prior->ncomp; ++g)
        for (int i = 0; i < nx; ++i) mean[i] += prior->w[g] / wsum * prior->mean[MS * g + i];
    KPrior kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.ncomp = prior->ncomp;
    for (int g = 0; g < prior->ncomp; ++g) {
        double C[MSQ], Ci[MSQ];
        load_square(prior->cov + MSQ * g, nx, C);
        const double det = mat_inv(Ci, C, nx);
        mat_copy(kp.Ci[g], Ci);
        kp.lw[g] = std::log(prior->w[g] / wsum) - 0.5 * (nx * std::log(2.0 * M_PI) + std::log(det));
        for (int i = 0; i < nx; ++i) kp.mean[g][i] = prior->mean[MS * g + i];
        const double wg = prior->w[g] / wsum;
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < nx; ++j)
                cov[i * MS + j] += wg * (C[i * MS + j] + (prior->mean[MS * g + i] - mean[i]) *
                                                             (prior->mean[MS * g + j] - mean[j]));
    }
    DevDesc hd;
    std::memset(&hd, 0, sizeof(hd));
    if (!design_grid_host(*model, f->Wnom, mean, cov, hd.g)) {
        pmf_destroy(f);
        return fail(PMF_E_INVALID, "prior covariance gives a degenerate grid");
    }
    hd.gn = hd.g;
    hd.l = 0;
    hd.pscale = 1.0;
    e = hipMemcpy(f->desc, &hd, sizeof(hd), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_prior(f->km, kp, f->desc, f->tab, f->buf[0], model->precision, st);
    if (e == hipSuccess) e = normalise_current(f, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        pmf_destroy(f);
        return hip_fail(e, "pmf_create");
    }
    *out = f;
    return PMF_OK;
}

void pmf_destroy(pmf_filter* f) {
    if (!f) return;
    pmf_ctx* ctx = f->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 4; ++i) ctx_free(ctx, f->buf[i], nullptr);
    ctx_free(ctx, f->cbuf, nullptr);
    ctx_free(ctx, f->part, nullptr);
    ctx_free(ctx, f->bfac, nullptr);
    ctx_free(ctx, f->coef, nullptr);
    ctx_free(ctx, f->W, nullptr);
    ctx_free(ctx, f->tab, nullptr);
    ctx_free(ctx, f->desc, nullptr);
    ctx_free(ctx, f->D1, nullptr);
    ctx_free(ctx, f->D2, nullptr);
    for (int i = 0; i < 5; ++i) ctx_free(ctx, f->rk[i], nullptr);
    ctx_free(ctx, f->dconst, nullptr);
    batch_forget_filter(ctx, f);
    delete f;
}

pmf_status pmf_predict(pmf_filter* f, double T, void* stream) {
    if (!f) return fail(PMF_E_INVALID, "filter is NULL");
    if (!std::isfinite(T) || T < 0.0) return fail(PMF_E_INVALID, "T must be finite and >= 0");
    if (T == 0.0) return PMF_OK;
    if (f->in_batch) {
        hipError_t eb = batch_leave(f);
        if (eb != hipSuccess) return hip_fail(eb, "leave batch mode");
    }
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const PredictArgs& pa = predict_args(f, T);
    e = launch_plan(pa, f->desc, f->coef, st);
    if (e != hipSuccess) return hip_fail(e, "plan");
    if (f->model.integrator == PMF_INT_FDM || f->model.integrator == PMF_INT_SINE) {
        const int sine = f->model.integrator == PMF_INT_SINE ? 1 : 0;
        double trA = 0.0;
        for (int i = 0; i < f->model.nx; ++i) trA += pa.A[i * MS + i];
        void* t1 = f->buf[(f->cur + 1) % 4];
        void* t2 = f->buf[(f->cur + 2) % 4];
        if (f->es == sizeof(double))
            e = launch_predict_fdm<double>(f->km, f->desc, f->coef, static_cast<double*>(f->buf[f->cur]),
                                           static_cast<double*>(t1), static_cast<double*>(t2), trA, sine, st);
        else
            e = launch_predict_fdm<float>(f->km, f->desc, f->coef, static_cast<float*>(f->buf[f->cur]),
                                          static_cast<float*>(t1), static_cast<float*>(t2), trA, sine, st);
        if (e != hipSuccess) return hip_fail(e, "predict (finite differences)");
        return PMF_OK;
    }
    if (f->model.grid == PMF_GRID_FOURIER) {
        if (f->es == sizeof(double))
            e = launch_predict_fourier<double>(f->km, f->desc, f->coef, f->cbuf, static_cast<double*>(f->buf[f->cur]), st);
        else
            e = launch_predict_fourier<float>(f->km, f->desc, f->coef, f->cbuf, static_cast<float*>(f->buf[f->cur]), st);
        if (e != hipSuccess) return hip_fail(e, "predict");
        return PMF_OK;
    }
    return cheb_predict(f, st);
}

pmf_status pmf_update(pmf_filter* f, const double* z, double* loglik, void* stream) {
    if (!f || !z) return fail(PMF_E_INVALID, "filter/z is NULL");
    for (int i = 0; i < f->model.nz; ++i)
        if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
    if (f->in_batch) {
        hipError_t eb = batch_leave(f);
        if (eb != hipSuccess) return hip_fail(eb, "leave batch mode");
    }
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int cur = f->cur, p = (cur + 1) % 4, q = (cur + 2) % 4, r = (cur + 3) % 4;
    if (f->es == sizeof(double)) {
        double** b = reinterpret_cast<double**>(f->buf);
        e = launch_like<double>(f->km, f->desc, f->tab, z, b[cur], b[p], f->part, f->nb, f->chunk, 1, st);
        if (e == hipSuccess) e = launch_update_finalize(f->km, f->desc, f->part, f->nb, f->bfac, st);
        if (e == hipSuccess) e = launch_scale_blocks<double>(b[p], f->ntot, f->chunk, f->bfac, st);
        if (e == hipSuccess)
            e = launch_interp<double>(f->km, f->desc, f->tab, f->W, b[p], b[q], b[r], f->part, f->nb, f->chunk, st);
        if (e == hipSuccess) e = launch_final_scale<double>(b[r], b[cur], f->ntot, f->desc, st);
    } else {
        float** b = reinterpret_cast<float**>(f->buf);
        e = launch_like<float>(f->km, f->desc, f->tab, z, b[cur], b[p], f->part, f->nb, f->chunk, 1, st);
        if (e == hipSuccess) e = launch_update_finalize(f->km, f->desc, f->part, f->nb, f->bfac, st);
        if (e == hipSuccess) e = launch_scale_blocks<float>(b[p], f->ntot, f->chunk, f->bfac, st);
        if (e == hipSuccess)
            e = launch_interp<float>(f->km, f->desc, f->tab, f->W, b[p], b[q], b[r], f->part, f->nb, f->chunk, st);
        if (e == hipSuccess) e = launch_final_scale<float>(b[r], b[cur], f->ntot, f->desc, st);
    }
    if (e != hipSuccess) return hip_fail(e, "update");
    f->cur = r;
    if (loglik) {
        e = hipMemcpyAsync(loglik, &f->desc->loglik, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "loglik copy");
    }
    return PMF_OK;
}

pmf_status pmf_sync_status(pmf_filter* f, void* stream) {
    if (!f) return fail(PMF_E_INVALID, "filter is NULL");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "sync");
    return take_status(f);
}

pmf_status pmf_moments(pmf_filter* f, double* mean, double* cov, void* stream) {
    if (!f || !mean || !cov) return fail(PMF_E_INVALID, "NULL argument");
    if (f->in_batch) {
        hipError_t eb = batch_leave(f);
        if (eb != hipSuccess) return hip_fail(eb, "leave batch mode");
    }
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (f->es == sizeof(double))
        e = launch_like<double>(f->km, f->desc, f->tab, nullptr, static_cast<double*>(f->buf[f->cur]), nullptr,
                                f->part, f->nb, f->chunk, 0, st);
    else
        e = launch_like<float>(f->km, f->desc, f->tab, nullptr, static_cast<float*>(f->buf[f->cur]), nullptr,
                               f->part, f->nb, f->chunk, 0, st);
    if (e == hipSuccess) e = launch_sums_finalize(f->km, f->desc, f->part, f->nb, f->bfac, st);
    DevDesc hd;
    if (e == hipSuccess) e = hipMemcpyAsync(&hd, f->desc, sizeof(hd), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "moments");
    const int nx = f->model.nx;
    for (int i = 0; i < nx; ++i) {
        mean[i] = hd.mean[i];
        for (int j = 0; j < nx; ++j) cov[i * nx + j] = hd.cov[i * MS + j];
    }
    return take_status(f);
}

pmf_status pmf_last_substeps(pmf_filter* f, int* l) {
    if (!f || !l) return fail(PMF_E_INVALID, "NULL argument");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(l, &f->desc->l, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "substeps");
    return PMF_OK;
}

pmf_status pmf_get_state(pmf_filter* f, void* host_buf, size_t* bytes) {
    if (!f || !bytes) return fail(PMF_E_INVALID, "NULL argument");
    if (f->in_batch) {
        hipError_t eb = batch_leave(f);
        if (eb != hipSuccess) return hip_fail(eb, "leave batch mode");
    }
    const size_t need = sizeof(pmf_state_header) + (size_t)f->ntot * f->es;
    if (!host_buf) {
        *bytes = need;
        return PMF_OK;
    }
    if (*bytes < need) return fail(PMF_E_INVALID, "buffer too small");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    DevDesc hd;
    if (e == hipSuccess) e = hipMemcpy(&hd, f->desc, sizeof(hd), hipMemcpyDeviceToHost);
    unsigned char* out = static_cast<unsigned char*>(host_buf);
    if (e == hipSuccess)
        e = hipMemcpy(out + sizeof(pmf_state_header), f->buf[f->cur], (size_t)f->ntot * f->es, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_state");
    pmf_state_header h;
    std::memset(&h, 0, sizeof(h));
    h.magic = PMF_STATE_MAGIC;
    h.version = 2;
    h.nx = f->model.nx;
    h.grid = f->model.grid;
    h.precision = f->model.precision;
    h.status = hd.status;
    for (int a = 0; a < MS; ++a) h.N[a] = a < f->model.nx ? f->model.N[a] : 1;
    for (int a = 0; a < MS; ++a) h.c[a] = hd.g.c[a];
    mat_copy(h.M, hd.g.M);
    h.t = hd.t;
    std::memcpy(out, &h, sizeof(h));
    *bytes = need;
    return PMF_OK;
}

pmf_status pmf_set_state(pmf_filter* f, const void* host_buf, size_t bytes) {
    if (!f || !host_buf) return fail(PMF_E_INVALID, "NULL argument");
    if (f->in_batch) {
        hipError_t eb = batch_leave(f);
        if (eb != hipSuccess) return hip_fail(eb, "leave batch mode");
    }
    if (bytes < sizeof(pmf_state_header)) return fail(PMF_E_INVALID, "image too small");
    pmf_state_header h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (h.magic != PMF_STATE_MAGIC || h.version != 2) return fail(PMF_E_INVALID, "not a pmf state image");
    if (h.nx != f->model.nx || h.grid != f->model.grid || h.precision != f->model.precision)
        return fail(PMF_E_INVALID, "image of a different filter kind");
    for (int a = 0; a < f->model.nx; ++a)
        if (h.N[a] != f->model.N[a]) return fail(PMF_E_INVALID, "image of a different grid size");
    if (bytes < sizeof(h) + (size_t)f->ntot * f->es) return fail(PMF_E_INVALID, "image truncated");
    for (int i = 0; i < MSQ; ++i)
        if (!std::isfinite(h.M[i])) return fail(PMF_E_INVALID, "non-finite grid");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    DevDesc hd;
    if (e == hipSuccess) e = hipMemcpy(&hd, f->desc, sizeof(hd), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    for (int a = 0; a < MS; ++a) hd.g.c[a] = a < f->model.nx ? h.c[a] : 0.0;
    mat_zero(hd.g.M);
    for (int i = 0; i < f->model.nx; ++i)
        for (int j = 0; j < f->model.nx; ++j) hd.g.M[i * MS + j] = h.M[i * MS + j];
    grid_finish(hd.g, f->model.nx);
    if (!(hd.g.vol > 0.0)) return fail(PMF_E_INVALID, "singular grid matrix");
    hd.gn = hd.g;
    hd.t = h.t;
    hd.status = 0;
    hd.pscale = 1.0;
    e = hipMemcpy(f->desc, &hd, sizeof(hd), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(f->buf[f->cur], static_cast<const unsigned char*>(host_buf) + sizeof(h), (size_t)f->ntot * f->es,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    return PMF_OK;
}

void* pmf_density_ptr(pmf_filter* f) {
    if (!f) return nullptr;
    if (f->in_batch && batch_leave(f) != hipSuccess) return nullptr;
    return f->buf[f->cur];
}

pmf_status pmf_stream_sync(void* stream) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return PMF_OK;
}

}  // extern "C"

namespace pmf {

hipError_t normalise_current(pmf_filter* f, hipStream_t st) {
    hipError_t e;
    if (f->es == sizeof(double)) {
        double* P = static_cast<double*>(f->buf[f->cur]);
        e = launch_like<double>(f->km, f->desc, f->tab, nullptr, P, nullptr, f->part, f->nb, f->chunk, 0, st);
        if (e == hipSuccess) e = launch_sums_finalize(f->km, f->desc, f->part, f->nb, f->bfac, st);
        if (e == hipSuccess) e = launch_scale_blocks<double>(P, f->ntot, f->chunk, f->bfac, st);
    } else {
        float* P = static_cast<float*>(f->buf[f->cur]);
        e = launch_like<float>(f->km, f->desc, f->tab, nullptr, P, nullptr, f->part, f->nb, f->chunk, 0, st);
        if (e == hipSuccess) e = launch_sums_finalize(f->km, f->desc, f->part, f->nb, f->bfac, st);
        if (e == hipSuccess) e = launch_scale_blocks<float>(P, f->ntot, f->chunk, f->bfac, st);
    }
    return e;
}

pmf_status take_status(pmf_filter* f) {
    int stw = 0;
    hipError_t e = hipMemcpy(&stw, &f->desc->status, sizeof(int), hipMemcpyDeviceToHost);
    const int zero = 0;
    if (e == hipSuccess) e = hipMemcpy(&f->desc->status, &zero, sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "status");
    if (stw & PMF_E_DEGENERATE) {
        g_last_error = "a measurement update met a degenerate normaliser; it left the filter unchanged";
        return (pmf_status)(stw & (PMF_E_DEGENERATE | PMF_W_BOUNDARY | PMF_E_INVALID));
    }
    if (stw & PMF_E_INVALID) {
        g_last_error = "a predict needed more than 4096 substeps";
        return PMF_E_INVALID;
    }
    return (pmf_status)(stw & PMF_W_BOUNDARY);
}

const PredictArgs& predict_args(pmf_filter* f, double T) {
    if (f->have_pa && f->pa.T == T) return f->pa;
    PredictArgs& a = f->pa;
    std::memset(&a, 0, sizeof(a));
    const int n = f->model.nx;
    a.T = T;
    load_square(f->model.A, n, a.A);
    diffusion(f->model, a.D);
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += a.A[i * MS + i];
    a.etr = std::exp(-tr * T);
    expm3(a.Phi, a.A, T, n);
    expm3(a.emh, a.A, -0.5 * T, n);
    expm3(a.emT, a.A, -T, n);
    w_integral(a.W, a.A, a.D, T, n);
    a.lmin = f->model.substeps;
    a.integ = f->model.integrator;
    a.nx = n;
    a.lmax = LMAX;
    for (int i = 0; i < MS; ++i) a.rho[i] = f->km.rho[i];
    f->have_pa = true;
    return a;
}

pmf_status cheb_predict(pmf_filter* f, hipStream_t st) {
    // the substep count is decided on the device from the current grid: read it
    int l = 0;
    hipError_t e = hipMemcpyAsync(&l, &f->desc->l, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "substep count");
    if (f->es == sizeof(float) && cheb_mfma_available(f)) {
        return cheb_predict_mfma(f, l, st);
    }
    auto run = [&](auto* q, auto* y, auto* kf, auto* acc, auto* t1, auto* t2, auto* D1, auto* D2) -> hipError_t {
        using T = std::remove_pointer_t<decltype(q)>;
        hipError_t err = hipSuccess;
        for (int n = 0; n < l && err == hipSuccess; ++n) {
            const int ks[4] = {2 * n, 2 * n + 1, 2 * n + 1, 2 * n + 2};
            for (int stg = 1; stg <= 4 && err == hipSuccess; ++stg) {
                const T* in = (stg == 1) ? q : y;
                err = launch_cheb_rhs<T>(f->km, D1, D2, f->coef, ks[stg - 1], in, kf, t1, t2, st);
                if (err == hipSuccess) err = launch_rk4_stage<T>(q, y, kf, acc, f->ntot, f->desc, stg, st);
            }
        }
        if (err == hipSuccess) err = launch_scale_etr<T>(q, f->ntot, f->desc, st);
        return err;
    };
    if (f->es == sizeof(double)) {
        double** r = reinterpret_cast<double**>(f->rk);
        e = run(static_cast<double*>(f->buf[f->cur]), r[0], r[1], r[2], r[3], r[4],
                static_cast<const double*>(f->D1), static_cast<const double*>(f->D2));
    } else {
        float** r = reinterpret_cast<float**>(f->rk);
        e = run(static_cast<float*>(f->buf[f->cur]), r[0], r[1], r[2], r[3], r[4], static_cast<const float*>(f->D1),
                static_cast<const float*>(f->D2));
    }
    if (e != hipSuccess) return hip_fail(e, "chebyshev predict");
    return PMF_OK;
}

}  // namespace pmf
