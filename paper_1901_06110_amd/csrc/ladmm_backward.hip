// Reverse mode through unrolled linearized PnP-ADMM (Section 2, Algorithm 1)
// with per-iteration checkpoints.
//
// Iteration k maps (x, v, u) -> (x', v', u'):
//   q  = mu (alpha x + rho (v - u) - grad f(x)),  x' = Pi_C(q)
//   z  = x' + u,  v' = W_k z,  u' = u + x' - v'
// with W_k = W(z_k, h) while k <= k0 and W(z_{k0}, h) afterwards.  Given the
// adjoints (xb, vb, ub) of (x', v', u'), one reverse step computes
//   vt = vb - ub                             (adjoint of v' through v' and u')
//   zb = W vt,  gb = d<vt, W(g) z>/dg,  hb   (DSG-NLM backward; W symmetric)
//   xt = xb + ub + zb (+ gb when the guide is z itself)
//   qb = xt on the open box, 0 elsewhere
//   xb_prev = mu (alpha qb - H(x) qb)        (H = A^T A for SR, diag phi'' for SPI)
//   vb_prev = mu rho qb,  ub_prev = ub + zb (+ gb) - mu rho qb
//   rhob   += sum qb mu (v - u - q)          (explicit dependence on rho)
// The adjoint of the frozen guide z_{k0} accumulates over k > k0 and joins
// z's adjoint at iteration k0.  Reductions are fixed-order (per-block
// partials, then one block), so runs are bit-reproducible.
#include <cmath>

#include "internal.h"

namespace dsnlm {

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out);
ImgDesc base_desc(const dsnlm_weights* w);

namespace {

inline int nblk(size_t n) { return (int)((n + 255) / 256); }

// vt = vb - ub
__global__ void __launch_bounds__(256) k_vt(const float* __restrict__ vb, const float* __restrict__ ub,
                                           float* __restrict__ vt, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) vt[i] = vb[i] - ub[i];
}

struct RevArgs {
    const float* x;      // x_{k-1}
    const float* v;      // v_{k-1}
    const float* u;      // u_{k-1}
    const float* xk;     // x_k
    const float* zb;     // W vt
    const float* gb;     // guide adjoint of this iteration (guide = z_k), or null
    const float* gacc;   // accumulated frozen-guide adjoint joining at k0, or null
    const unsigned char* ones;  // SPI counts (null for SR)
    float* xb;           // in: adjoint of x_k; out: adjoint of x_{k-1}
    float* vb;           // out: adjoint of v_{k-1}
    float* ub;           // in: adjoint of u_k; out: adjoint of u_{k-1}
    float* qb;           // out: masked adjoint of q (SR needs A^T A qb next)
    float* partials;     // per-block sums for rhob
    int n;
    float alpha, rho, mu, lo, hi;
    float eta_over_K, K, t_min;
    int spi;
};

// Everything of the reverse step except the SR Hessian term.
__global__ void __launch_bounds__(256) k_rev(RevArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    float part = 0.f;
    if (i < a.n) {
        float zt = a.zb[i];
        if (a.gb) zt += a.gb[i];
        if (a.gacc) zt += a.gacc[i];
        const float ubk = a.ub[i];
        const float xt = a.xb[i] + ubk + zt;
        const float xk = a.xk[i];
        const bool inside = xk > a.lo && xk < a.hi;
        const float qb = inside ? xt : 0.f;
        const float mrq = a.mu * a.rho * qb;
        a.vb[i] = mrq;
        a.ub[i] = ubk + zt - mrq;
        a.qb[i] = qb;
        float hq = 0.f;
        if (a.spi) {
            // phi''(t) = (eta/K)^2 K1 e / (1 - e)^2, e = exp(-eta t / K), t > t_min
            const float t = a.x[i];
            if (t > a.t_min) {
                const float s = a.eta_over_K * t;
                const float e = expf(-s);
                const float om = -expm1f(-s);
                hq = a.eta_over_K * a.eta_over_K * (float)a.ones[i] * e / (om * om) * qb;
            }
            a.xb[i] = a.mu * (a.alpha * qb - hq);
        }
        // explicit rho dependence: dq/drho = mu (v - u - q); q = x_k where qb != 0
        part = qb * a.mu * (a.v[i] - a.u[i] - xk);
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[blockIdx.x] = (float)sh[0];
}

// SR: xb = mu (alpha qb - A^T A qb), with hq = A^T A qb precomputed.
__global__ void __launch_bounds__(256) k_rev_sr(const float* __restrict__ qb, const float* __restrict__ hq,
                                               float* __restrict__ xb, int n, float mu, float alpha) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) xb[i] = mu * (alpha * qb[i] - hq[i]);
}

// dparams[0] += sum of partials (rhob), dparams[1] += *dh (hb); fixed order.
__global__ void __launch_bounds__(256) k_accum_params(const float* __restrict__ partials, int nb,
                                                     const float* __restrict__ dh, float* __restrict__ dparams) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) acc += partials[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dparams[0] += (float)sh[0];
        if (dh) dparams[1] += *dh;
    }
}

// acc += g
__global__ void __launch_bounds__(256) k_axpy1(float* __restrict__ acc, const float* __restrict__ g, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) acc[i] += g[i];
}

}  // namespace

// SR helpers from ladmm.hip: r = A x (y null) and g = A^T r.
int sr_apply_AtA(const ladmm_operator* op, const float* x, float* lr, float* out, hipStream_t st);

}  // namespace dsnlm

using namespace dsnlm;

extern "C" int ladmm_step_backward(const ladmm_operator* op, const ladmm_params* p, int k, const float* guide,
                                   const float* x_prev, const float* v_prev, const float* u_prev,
                                   const float* x_k, const float* z_k, float* xbar, float* vbar, float* ubar,
                                   float* gacc, float* dparams, void* stream) {
    if (!op || !p || !guide || !x_prev || !v_prev || !u_prev || !x_k || !z_k || !xbar || !vbar || !ubar ||
        !dparams)
        return fail(DSNLM_EINVAL, "ladmm_step_backward: null pointer");
    if (k < 1) return fail(DSNLM_EINVAL, "ladmm_step_backward: k is 1-based");
    if (p->denoiser != 0) return fail(DSNLM_EUNSUPPORTED, "ladmm_step_backward: DSG-NLM denoiser only");
    if (k > p->freeze_after && !gacc)
        return fail(DSNLM_EINVAL, "ladmm_step_backward: frozen iterations need the guide-adjoint accumulator");
    const int n1 = op->n1, n2 = op->n2;
    if (n1 < 1 || n2 < 1) return fail(DSNLM_EINVAL, "ladmm_step_backward: bad image size");
    const float h = p->h > 0.f ? p->h : std::sqrt(p->lambda / p->rho);
    int rc = check_denoiser_args(n1, n2, p->S, p->P, h, "ladmm_step_backward");
    if (rc) return rc;
    if (!(p->lambda > 0.f) || !(p->rho > 0.f) || !(p->gamma > 0.f) || !(p->lo < p->hi))
        return fail(DSNLM_EINVAL, "ladmm_step_backward: bad parameters");
    if (op->kind == LADMM_OP_SR) {
        if (!op->taps || op->blur_size < 1 || op->blur_size > 31 || op->blur_size % 2 == 0 || op->factor < 1 ||
            op->factor > 8 || (op->blur_size - 1) / 2 >= (n1 < n2 ? n1 : n2))
            return fail(DSNLM_EINVAL, "ladmm_step_backward: bad super-resolution operator");
    } else if (op->kind == LADMM_OP_SPI) {
        if (!op->ones || op->K < 1 || !(op->eta > 0.f) || !(op->t_min > 0.f))
            return fail(DSNLM_EINVAL, "ladmm_step_backward: bad single-photon operator");
    } else {
        return fail(DSNLM_EINVAL, "ladmm_step_backward: unknown operator kind");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)n1 * n2;
    dsnlm_weights* w = nullptr;
    float* scratch = nullptr;
    const size_t mlr = op->kind == LADMM_OP_SR
                           ? (size_t)((n1 + op->factor - 1) / op->factor) * ((n2 + op->factor - 1) / op->factor)
                           : 0;
    // layout: y | vt | zb | gb | qb | hq | lr | partials | dh
    const size_t need = 6 * n + mlr + nblk(n) + 8;
    rc = check_hip(hipMalloc(&scratch, need * sizeof(float)), "ladmm_step_backward scratch");
    if (rc) return rc;
    float* y = scratch;
    float* vt = y + n;
    float* zb = vt + n;
    float* gb = zb + n;
    float* qb = gb + n;
    float* hq = qb + n;
    float* lr = hq + n;
    float* partials = lr + mlr;
    float* dh = partials + nblk(n);
    // recompute the forward denoiser of iteration k: W(guide) applied to z_k
    rc = dsnlm_forward(guide, z_k, y, n1, n2, p->S, p->P, h, stream, &w);
    if (!rc) {
        hipLaunchKernelGGL(k_vt, dim3(nblk(n)), dim3(256), 0, st, vbar, ubar, vt, (int)n);
        rc = check_hip(hipGetLastError(), "reverse step");
    }
    const bool adaptive = k <= p->freeze_after;
    if (!rc) rc = dsnlm_apply_backward(w, z_k, vt, zb, gb, dh, stream);
    if (!rc) {
        const float alpha = 1.0f / p->gamma;
        RevArgs a{};
        a.x = x_prev;
        a.v = v_prev;
        a.u = u_prev;
        a.xk = x_k;
        a.zb = zb;
        a.gb = adaptive ? gb : nullptr;
        a.gacc = (k == p->freeze_after) ? gacc : nullptr;
        a.ones = op->kind == LADMM_OP_SPI ? op->ones : nullptr;
        a.xb = xbar;
        a.vb = vbar;
        a.ub = ubar;
        a.qb = qb;
        a.partials = partials;
        a.n = (int)n;
        a.alpha = alpha;
        a.rho = p->rho;
        a.mu = 1.0f / (alpha + p->rho);
        a.lo = p->lo;
        a.hi = p->hi;
        a.spi = op->kind == LADMM_OP_SPI;
        if (a.spi) {
            a.eta_over_K = op->eta / (float)op->K;
            a.K = (float)op->K;
            a.t_min = op->t_min;
        }
        ProfScope prof(DSNLM_K_LADMM, st);
        if (!adaptive) hipLaunchKernelGGL(k_axpy1, dim3(nblk(n)), dim3(256), 0, st, gacc, gb, (int)n);
        hipLaunchKernelGGL(k_rev, dim3(nblk(n)), dim3(256), 0, st, a);
        rc = check_hip(hipGetLastError(), "reverse step");
        if (!rc && !a.spi) {
            rc = sr_apply_AtA(op, qb, lr, hq, st);
            if (!rc) {
                hipLaunchKernelGGL(k_rev_sr, dim3(nblk(n)), dim3(256), 0, st, qb, hq, xbar, (int)n, a.mu, alpha);
                rc = check_hip(hipGetLastError(), "reverse step");
            }
        }
        if (!rc) {
            hipLaunchKernelGGL(k_accum_params, dim3(1), dim3(256), 0, st, partials, nblk(n), dh, dparams);
            rc = check_hip(hipGetLastError(), "reverse step");
        }
    }
    // free only after the queued work has consumed the scratch and the handle
    hipError_t e = hipStreamSynchronize(st);
    if (!rc) rc = check_hip(e, "reverse step synchronise");
    (void)hipFree(scratch);
    dsnlm_weights_destroy(w);
    return rc;
}

extern "C" int ladmm_solve_backward(const ladmm_operator* op, const ladmm_params* p, const float* x0,
                                    const float* v0, const float* u0, const float* checkpoints, float* xbar,
                                    float* vbar, float* ubar, float* dparams, void* stream) {
    if (!op || !p || !x0 || !v0 || !u0 || !checkpoints || !xbar || !vbar || !ubar || !dparams)
        return fail(DSNLM_EINVAL, "ladmm_solve_backward: null pointer");
    if (p->iters < 1) return DSNLM_OK;
    if (p->freeze_after < 1) return fail(DSNLM_EINVAL, "ladmm_solve_backward: freeze_after must be >= 1");
    if (p->denoiser != 0) return fail(DSNLM_EUNSUPPORTED, "ladmm_solve_backward: DSG-NLM denoiser only");
    const size_t n = (size_t)op->n1 * op->n2;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* gacc = nullptr;
    int rc = DSNLM_OK;
    if (p->iters > p->freeze_after) {
        rc = check_hip(hipMalloc(&gacc, n * sizeof(float)), "guide adjoint");
        if (!rc) rc = check_hip(hipMemsetAsync(gacc, 0, n * sizeof(float), st), "guide adjoint");
        if (rc) return rc;
    }
    auto ck = [&](int k, int which) { return checkpoints + (4 * (size_t)(k - 1) + which) * n; };
    const int k0 = p->freeze_after < p->iters ? p->freeze_after : p->iters;
    for (int k = p->iters; k >= 1 && !rc; --k) {
        const float* xp = k > 1 ? ck(k - 1, 0) : x0;
        const float* vp = k > 1 ? ck(k - 1, 1) : v0;
        const float* up = k > 1 ? ck(k - 1, 2) : u0;
        const float* guide = k <= k0 ? ck(k, 3) : ck(k0, 3);
        rc = ladmm_step_backward(op, p, k, guide, xp, vp, up, ck(k, 0), ck(k, 3), xbar, vbar, ubar, gacc, dparams,
                                 stream);
    }
    if (gacc) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(gacc);
    }
    return rc;
}
