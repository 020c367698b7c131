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
#include <mutex>
#include <string>

#include "internal.h"

namespace dsnlm {

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out);
ImgDesc base_desc(const dsnlm_weights* w);
// SR helper from ladmm.hip: out = A^T A x (lr: low-resolution scratch).
int sr_apply_AtA(const ladmm_operator* op, const float* x, float* lr, float* out, hipStream_t st);

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

// v[0 .. n) = 0 (a kernel rather than a memset, so the sequence stays
// capturable into a graph)
__global__ void __launch_bounds__(256) k_zero(float* __restrict__ v, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = 0.f;
}

// The end of the reverse pass: the adjoint of the initial image when
// Algorithm 1 starts from x0 = v0 (dinit = xbar + vbar), and the parameter
// derivatives.  dparams: [0] explicit d/drho, [1] d/dh on entry; [2] d/dlambda
// and [3] d/drho on return, through h = sqrt(lambda / rho) when coupled.
__global__ void __launch_bounds__(256) k_rev_final(const float* __restrict__ xb, const float* __restrict__ vb,
                                                  float* __restrict__ dinit, int n, float* __restrict__ dparams,
                                                  float h, float lambda, float rho, int coupled) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (dinit && i < n) dinit[i] = xb[i] + vb[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const float drho_x = dparams[0], dh = dparams[1];
        dparams[2] = coupled ? dh * h / (2.0f * lambda) : 0.f;
        dparams[3] = coupled ? drho_x - dh * h / (2.0f * rho) : drho_x;
    }
}

// Reverse-pass workspace of one device (grow-only, reused by every call):
// the weights rebuilt for adaptive iterations, the frozen weights, and the
// per-step scratch.
struct RevWorkspace {
    dsnlm_weights* wa = nullptr;
    dsnlm_weights* wf = nullptr;
    float* scratch = nullptr;
    size_t cap = 0;
};
constexpr int kRevDevices = 64;
std::mutex g_rev_mu;
RevWorkspace g_rev[kRevDevices];

// Scratch layout: y | vt | zb | gb | qb | hq | gacc | lr | partials | dh
struct RevScratch {
    float *y, *vt, *zb, *gb, *qb, *hq, *lr, *partials, *dh, *gacc;
};

int rev_scratch(RevWorkspace& ws, size_t n, size_t mlr, RevScratch* r) {
    const size_t need = 7 * n + mlr + nblk(n) + 64;
    if (ws.cap < need) {
        if (ws.scratch) {
            (void)hipDeviceSynchronize();  // a previous call may still read it
            (void)hipFree(ws.scratch);
        }
        ws.scratch = nullptr;
        ws.cap = 0;
        int rc = check_hip(hipMalloc(&ws.scratch, need * sizeof(float)), "reverse-pass scratch");
        if (rc) return rc;
        ws.cap = need;
    }
    float* b = ws.scratch;
    r->y = b;
    r->vt = b + n;
    r->zb = b + 2 * n;
    r->gb = b + 3 * n;
    r->qb = b + 4 * n;
    r->hq = b + 5 * n;
    r->gacc = b + 6 * n;
    r->lr = b + 7 * n;
    r->partials = r->lr + mlr;
    r->dh = r->partials + nblk(n);
    return DSNLM_OK;
}

// A handle of the workspace for an n1 x n2 image (one of another size is
// dropped after the device has finished with it).
int rev_handle(dsnlm_weights** w, int n1, int n2) {
    if (*w && ((*w)->n1 != n1 || (*w)->n2 != n2)) {
        (void)hipDeviceSynchronize();
        dsnlm_weights_destroy(*w);
        *w = nullptr;
    }
    return DSNLM_OK;
}

int check_rev_args(const ladmm_operator* op, const ladmm_params* p, const char* who, float* h_out) {
    std::string w(who);
    if (!op || !p) return fail(DSNLM_EINVAL, w + ": null pointer");
    if (p->denoiser != 0) return fail(DSNLM_EUNSUPPORTED, w + ": DSG-NLM denoiser only");
    const int n1 = op->n1, n2 = op->n2;
    if (n1 < 1 || n2 < 1) return fail(DSNLM_EINVAL, w + ": bad image size");
    if (!(p->lambda > 0.f) || !(p->rho > 0.f) || !(p->gamma > 0.f) || !(p->lo < p->hi) || p->freeze_after < 1)
        return fail(DSNLM_EINVAL, w + ": bad parameters");
    const float h = p->h > 0.f ? p->h : std::sqrt(p->lambda / p->rho);
    int rc = check_denoiser_args(n1, n2, p->S, p->P, h, who);
    if (rc) return rc;
    if (op->kind == LADMM_OP_SR) {
        if (!op->taps || op->blur_size < 1 || op->blur_size > 31 || op->blur_size % 2 == 0 || op->factor < 1 ||
            op->factor > 8 || (op->blur_size - 1) / 2 >= (n1 < n2 ? n1 : n2))
            return fail(DSNLM_EINVAL, w + ": bad super-resolution operator");
    } else if (op->kind == LADMM_OP_SPI) {
        if (!op->ones || op->K < 1 || !(op->eta > 0.f) || !(op->t_min > 0.f))
            return fail(DSNLM_EINVAL, w + ": bad single-photon operator");
    } else {
        return fail(DSNLM_EINVAL, w + ": unknown operator kind");
    }
    *h_out = h;
    return DSNLM_OK;
}

// One reverse step k (see the top of the file).  w holds the weights of the
// iteration: rebuilt here from `guide` when `rebuild`, else the frozen weights
// already built (only the apply for z_k is redone, which the backward needs).
// `adaptive`: the guide of iteration k is z_k itself, so its adjoint joins z's.
int enqueue_rev_step(const ladmm_operator* op, const ladmm_params* p, float h, int k, dsnlm_weights** w,
                     bool rebuild, bool adaptive, const float* guide, const float* x_prev, const float* v_prev,
                     const float* u_prev, const float* x_k, const float* z_k, float* xbar, float* vbar,
                     float* ubar, const float* gacc_join, float* gacc_add, float* dparams, const RevScratch& r,
                     hipStream_t st) {
    const int n1 = op->n1, n2 = op->n2;
    const size_t n = (size_t)n1 * n2;
    void* stream = st;
    int rc = rebuild ? dsnlm_forward(guide, z_k, r.y, n1, n2, p->S, p->P, h, stream, w)
                     : dsnlm_apply(*w, z_k, r.y, stream);
    if (!rc) {
        hipLaunchKernelGGL(k_vt, dim3(nblk(n)), dim3(256), 0, st, vbar, ubar, r.vt, (int)n);
        rc = check_hip(hipGetLastError(), "reverse step");
    }
    if (!rc) rc = dsnlm_apply_backward(*w, z_k, r.vt, r.zb, r.gb, r.dh, stream);
    if (rc) return rc;
    const float alpha = 1.0f / p->gamma;
    RevArgs a{};
    a.x = x_prev;
    a.v = v_prev;
    a.u = u_prev;
    a.xk = x_k;
    a.zb = r.zb;
    a.gb = adaptive ? r.gb : nullptr;
    a.gacc = gacc_join;
    a.ones = op->kind == LADMM_OP_SPI ? op->ones : nullptr;
    a.xb = xbar;
    a.vb = vbar;
    a.ub = ubar;
    a.qb = r.qb;
    a.partials = r.partials;
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
    if (gacc_add) hipLaunchKernelGGL(k_axpy1, dim3(nblk(n)), dim3(256), 0, st, gacc_add, r.gb, (int)n);
    hipLaunchKernelGGL(k_rev, dim3(nblk(n)), dim3(256), 0, st, a);
    rc = check_hip(hipGetLastError(), "reverse step");
    if (!rc && !a.spi) {
        rc = sr_apply_AtA(op, r.qb, r.lr, r.hq, st);
        if (!rc) {
            hipLaunchKernelGGL(k_rev_sr, dim3(nblk(n)), dim3(256), 0, st, r.qb, r.hq, xbar, (int)n, a.mu, alpha);
            rc = check_hip(hipGetLastError(), "reverse step");
        }
    }
    if (!rc) {
        hipLaunchKernelGGL(k_accum_params, dim3(1), dim3(256), 0, st, r.partials, nblk(n), r.dh, dparams);
        rc = check_hip(hipGetLastError(), "reverse step");
    }
    return rc;
}

size_t lr_floats(const ladmm_operator* op) {
    return op->kind == LADMM_OP_SR
               ? (size_t)((op->n1 + op->factor - 1) / op->factor) * ((op->n2 + op->factor - 1) / op->factor)
               : 0;
}

}  // namespace

}  // namespace dsnlm

using namespace dsnlm;

extern "C" int ladmm_step_backward(const ladmm_operator* op, const ladmm_params* p, int k, const float* guide,
                                   const float* x_prev, const float* v_prev, const float* u_prev,
                                   const float* x_k, const float* z_k, float* xbar, float* vbar, float* ubar,
                                   float* gacc, float* dparams, void* stream) {
    if (!guide || !x_prev || !v_prev || !u_prev || !x_k || !z_k || !xbar || !vbar || !ubar || !dparams)
        return fail(DSNLM_EINVAL, "ladmm_step_backward: null pointer");
    if (k < 1) return fail(DSNLM_EINVAL, "ladmm_step_backward: k is 1-based");
    float h;
    int rc = check_rev_args(op, p, "ladmm_step_backward", &h);
    if (rc) return rc;
    if (k > p->freeze_after && !gacc)
        return fail(DSNLM_EINVAL, "ladmm_step_backward: frozen iterations need the guide-adjoint accumulator");
    int dev = 0;
    rc = check_hip(hipGetDevice(&dev), "ladmm_step_backward: hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kRevDevices) return fail(DSNLM_EUNSUPPORTED, "ladmm_step_backward: device index too large");
    std::lock_guard<std::mutex> lk(g_rev_mu);
    RevWorkspace& ws = g_rev[dev];
    RevScratch r;
    rc = rev_scratch(ws, (size_t)op->n1 * op->n2, lr_floats(op), &r);
    if (!rc) rc = rev_handle(&ws.wa, op->n1, op->n2);
    if (rc) return rc;
    const bool adaptive = k <= p->freeze_after;
    // the weights are rebuilt from the guide (their input z_k while adaptive)
    return enqueue_rev_step(op, p, h, k, &ws.wa, true, adaptive, guide, x_prev, v_prev, u_prev, x_k, z_k, xbar, vbar, ubar,
                            k == p->freeze_after ? gacc : nullptr, adaptive ? nullptr : gacc, dparams, r,
                            static_cast<hipStream_t>(stream));
}

extern "C" int ladmm_solve_backward(const ladmm_operator* op, const ladmm_params* p, const float* x0,
                                    const float* v0, const float* u0, const float* checkpoints, float* xbar,
                                    float* vbar, float* ubar, float* dinit, float* dparams, void* stream) {
    if (!x0 || !v0 || !u0 || !checkpoints || !xbar || !vbar || !ubar || !dparams)
        return fail(DSNLM_EINVAL, "ladmm_solve_backward: null pointer");
    float h;
    int rc = check_rev_args(op, p, "ladmm_solve_backward", &h);
    if (rc) return rc;
    if (p->iters < 0) return fail(DSNLM_EINVAL, "ladmm_solve_backward: iters must be >= 0");
    int dev = 0;
    rc = check_hip(hipGetDevice(&dev), "ladmm_solve_backward: hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kRevDevices) return fail(DSNLM_EUNSUPPORTED, "ladmm_solve_backward: device index too large");
    const size_t n = (size_t)op->n1 * op->n2;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_rev_mu);
    RevWorkspace& ws = g_rev[dev];
    RevScratch r;
    rc = rev_scratch(ws, n, lr_floats(op), &r);
    if (!rc) rc = rev_handle(&ws.wa, op->n1, op->n2);
    if (!rc) rc = rev_handle(&ws.wf, op->n1, op->n2);
    if (rc) return rc;
    {
        ProfScope prof(DSNLM_K_LADMM, st);
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, dparams, 4);
        if (p->iters > p->freeze_after) hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(256), 0, st, r.gacc, (int)n);
        rc = check_hip(hipGetLastError(), "ladmm_solve_backward: clear");
    }
    auto ck = [&](int k, int which) { return checkpoints + (4 * (size_t)(k - 1) + which) * n; };
    const int k0 = p->freeze_after < p->iters ? p->freeze_after : p->iters;
    // the frozen weights W(z_k0) serve every k > k0: built once
    if (!rc && p->iters > k0)
        rc = dsnlm_build_weights(ck(k0, 3), op->n1, op->n2, p->S, p->P, h, stream, &ws.wf);
    for (int k = p->iters; k >= 1 && !rc; --k) {
        const float* xp = k > 1 ? ck(k - 1, 0) : x0;
        const float* vp = k > 1 ? ck(k - 1, 1) : v0;
        const float* up = k > 1 ? ck(k - 1, 2) : u0;
        const bool adaptive = k <= k0;
        rc = enqueue_rev_step(op, p, h, k, adaptive ? &ws.wa : &ws.wf, adaptive, adaptive, ck(k, 3), xp, vp, up, ck(k, 0),
                              ck(k, 3), xbar, vbar, ubar, k == k0 && p->iters > k0 ? r.gacc : nullptr,
                              adaptive ? nullptr : r.gacc, dparams, r, st);
    }
    if (!rc) {
        ProfScope prof(DSNLM_K_LADMM, st);
        hipLaunchKernelGGL(k_rev_final, dim3(nblk(n)), dim3(256), 0, st, xbar, vbar, dinit, (int)n, dparams, h,
                           p->lambda, p->rho, p->h > 0.f ? 0 : 1);
        rc = check_hip(hipGetLastError(), "ladmm_solve_backward: final");
    }
    return rc;
}
