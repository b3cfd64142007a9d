// lbm_io.hip -- initial state, read-outs and FP64 reductions (not per step).
// Every kernel covers all domains of a batch; a thread finds its domain from
// the node offsets.
#include "lbm_internal.hpp"

namespace lbm {

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_init(long N, long S, const DomDev *doms, const long *noff,
                                              int ndom, const int32_t *kof, const double *rho,
                                              const double *u, const double *cc, T *f0, T *g0,
                                              T *f1, T *g1) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    const int k = kof[n];
    if (k < 0) return;
    const DomDev &D = doms[find_dom(noff, ndom, n)];
    const double r = rho ? rho[n] : 1.0;
    const double ux = u ? u[3 * n] : 0.0, uy = u ? u[3 * n + 1] : 0.0, uz = u ? u[3 * n + 2] : 0.0;
    const double C = cc ? cc[n] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < L::Q; i++) {
        const double eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
        const double feq = L::w[i] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        f0[pidx(i, k, L::Q)] = T(feq - L::w[i] * D.rho0);
        f1[pidx(i, k, L::Q)] = T(0);
        if (!((D.smask >> i) & 1u)) continue;
        const long s = sol_slot(D.smask, i);
        const double geq = D.ws[i] * C * (1.0 + eu / D.cs2s);
        const int qs = __builtin_popcount(D.smask);
        g0[pidx(s, k, qs)] = T(geq - D.ws[i] * D.c_ref);
        g1[pidx(s, k, qs)] = T(0);
    }
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_fields(long N, long S, const DomDev *doms, const long *noff,
                                                int ndom, const int32_t *kof, const T *f, const T *g,
                                                const double *phi_in, double *rho, double *u,
                                                double *cc, double *phi, uint8_t *type) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    const int k = kof[n];
    const DomDev &D = doms[find_dom(noff, ndom, n)];
    double r = 0, jx = 0, jy = 0, jz = 0, C = 0;
    const bool sol = k < 0;
    if (!sol) {
        double dr = 0, dc = 0;
        for (int i = 0; i < L::Q; i++) {
            const double fi = (double)f[pidx(i, k, L::Q)];
            dr += fi;
            jx += L::ex[i] * fi;
            jy += L::ey[i] * fi;
            jz += L::ez[i] * fi;
            if ((D.smask >> i) & 1u) dc += (double)g[pidx(sol_slot(D.smask, i), k, __builtin_popcount(D.smask))];
        }
        r = D.rho0 + dr;
        C = D.c_ref + dc;
    }
    if (rho) rho[n] = r;
    if (u) {
        u[3 * n] = sol ? 0.0 : (jx - 0.5 * D.F[0]) / r;
        u[3 * n + 1] = sol ? 0.0 : (jy - 0.5 * D.F[1]) / r;
        u[3 * n + 2] = sol ? 0.0 : (jz - 0.5 * D.F[2]) / r;
    }
    if (cc) cc[n] = C;
    if (phi) phi[n] = phi_in[n];
    if (type) type[n] = sol ? 1 : 0;
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_pops(long N, long S, const DomDev *doms, const long *noff,
                                              int ndom, const int32_t *kof, const T *f, const T *g,
                                              double *fo, double *go) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    const int k = kof[n];
    const DomDev &D = doms[find_dom(noff, ndom, n)];
    for (int i = 0; i < L::Q; i++) {
        if (fo) fo[i * N + n] = k < 0 ? 0.0 : (double)f[pidx(i, k, L::Q)] + L::w[i] * D.rho0;
        if (!go || !((D.smask >> i) & 1u)) continue;
        const long s = sol_slot(D.smask, i);
        go[s * N + n] = k < 0 ? 0.0 : (double)g[pidx(s, k, __builtin_popcount(D.smask))] + D.ws[i] * D.c_ref;
    }
}

__global__ __launch_bounds__(BLK) void k_zero_f64(double *p, long n) {
    const long i = (long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_zero_flag(int32_t *p) { *p = 0; }

template <typename T>
__global__ __launch_bounds__(BLK) void k_scatter_q(long nl, int Q, const T *lq, const int32_t *lnode,
                                                   const uint8_t *ldir, double *q) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    if (j < nl) q[(long)lnode[j] * Q + ldir[j]] = (double)lq[j];
}

// per-workgroup partial sums of C (fluid) and phi (all nodes), and a
// non-finite flag; the partials are then added in two fixed-order levels
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_diag(long N, long S, const DomDev *doms, const long *noff,
                                              int ndom, const int32_t *kof, const T *f, const T *g,
                                              const double *phi, double *part, int32_t *nan_flag) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    double cs = 0.0, ps = 0.0;
    int bad = 0;
    if (n < N) {
        ps = phi[n];
        const int k = kof[n];
        if (k >= 0) {
            const DomDev &D = doms[find_dom(noff, ndom, n)];
            double dc = 0.0;
            for (int i = 0; i < L::Q; i++) {
                const double fi = (double)f[pidx(i, k, L::Q)];
                if (!isfinite(fi)) bad = 1;
                if (!((D.smask >> i) & 1u)) continue;
                const double gi = (double)g[pidx(sol_slot(D.smask, i), k, __builtin_popcount(D.smask))];
                if (!isfinite(gi)) bad = 1;
                dc += gi;
            }
            cs = D.c_ref + dc;
        }
    }
    const double bc = block_sum(cs);
    const double bp = block_sum(ps);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bc;
        part[2 * blockIdx.x + 1] = bp;
    }
    if (bad) atomicOr(nan_flag, 1);
}

// the per-workgroup (C, phi) pairs of k_diag in two fixed-order levels:
// workgroup b of FOLD_G sums its contiguous share into bpart[2b], [2b + 1]
__global__ __launch_bounds__(BLK) void k_sum_pairs(const double *part, long nb, double *bpart) {
    const long len = (nb + FOLD_G - 1) / FOLD_G;
    const long lo = (long)blockIdx.x * len, hi = lo + len < nb ? lo + len : nb;
    double a = 0.0, b = 0.0;
    for (long j = lo + threadIdx.x; j < hi; j += BLK) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    a = block_sum(a);
    b = block_sum(b);
    if (threadIdx.x == 0) {
        bpart[2 * blockIdx.x] = a;
        bpart[2 * blockIdx.x + 1] = b;
    }
}

__global__ __launch_bounds__(BLK) void k_sum_parts(const double *part, long nb, double *out) {
    double a = 0.0, b = 0.0;
    for (long j = threadIdx.x; j < nb; j += BLK) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    a = block_sum(a);
    b = block_sum(b);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// Fixed-order sums in two levels: workgroup b of FOLD_G adds its contiguous
// share of the slots (lane stride, then the block reduction) into bpart[b];
// one workgroup then adds the FOLD_G partials in order.  The exchange slots
// are cleared as they are read.
__global__ __launch_bounds__(BLK) void k_fold_parts(double *part, long n, double *bpart) {
    const long len = (n + FOLD_G - 1) / FOLD_G;
    const long lo = (long)blockIdx.x * len, hi = lo + len < n ? lo + len : n;
    double a = 0.0;
    for (long j = lo + threadIdx.x; j < hi; j += BLK) {
        const double v = part[j];
        if (v != 0.0) {
            a += v;
            part[j] = 0.0;
        }
    }
    a = block_sum(a);
    if (threadIdx.x == 0) bpart[blockIdx.x] = a;
}

// acc[0] += the FOLD_G partials, in order
__global__ __launch_bounds__(BLK) void k_fold_total(const double *bpart, double *acc) {
    double a = threadIdx.x < FOLD_G ? bpart[threadIdx.x] : 0.0;
    a = block_sum(a);
    if (threadIdx.x == 0) acc[0] += a;
}

static void fold_into(Ctx &c, double *part, long n, double *acc) {
    hipLaunchKernelGGL(k_fold_parts, dim3(FOLD_G), dim3(BLK), 0, c.stream, part, n, c.fpart);
    hipLaunchKernelGGL(k_fold_total, dim3(1), dim3(BLK), 0, c.stream, (const double *)c.fpart, acc);
}

hipError_t launch_fold_exchange(Ctx &c) {
    fold_into(c, c.xpart, c.n_xpart, c.dacc);
    if (c.any_planes) {
        fold_into(c, c.xio, c.task_cap, c.dacc + 3);
        fold_into(c, c.xio + c.task_cap, c.task_cap, c.dacc + 4);
    }
    return hipGetLastError();
}

hipError_t launch_zero_exchange(Ctx &c) {
    hipLaunchKernelGGL(k_zero_f64, dim3((c.n_xpart + BLK - 1) / BLK), dim3(BLK), 0, c.stream, c.xpart,
                       c.n_xpart);
    hipLaunchKernelGGL(k_zero_f64, dim3((2 * c.task_cap + BLK - 1) / BLK), dim3(BLK), 0, c.stream, c.xio,
                       2 * c.task_cap);
    return hipGetLastError();
}

template <class L, typename T>
static hipError_t init_impl(Ctx &c, const double *rho, const double *u, const double *cc) {
    const long nb = (c.N + BLK - 1) / BLK;
    c.cur = 0;
    hipLaunchKernelGGL((k_init<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.doms,
                       c.dnode_off, c.ndom, c.kof, rho, u, cc, (T *)c.f[0], (T *)c.g[0],
                       (T *)c.f[1], (T *)c.g[1]);
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(BLK), 0, c.stream, c.dacc, 8);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_zero_exchange(c) : e;
}

hipError_t launch_init(Ctx &c, const double *rho, const double *u, const double *cc) {
    if (c.Q == 9) return c.fp64 ? init_impl<D2Q9, double>(c, rho, u, cc) : init_impl<D2Q9, float>(c, rho, u, cc);
    return c.fp64 ? init_impl<D3Q19, double>(c, rho, u, cc) : init_impl<D3Q19, float>(c, rho, u, cc);
}

template <class L, typename T>
static hipError_t fields_impl(Ctx &c, double *rho, double *u, double *cc, double *phi, uint8_t *type) {
    const long nb = (c.N + BLK - 1) / BLK;
    hipError_t e = launch_phi_flush(c);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fields<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.doms,
                       c.dnode_off, c.ndom, c.kof, (const T *)c.f[c.cur], (const T *)c.g[c.cur],
                       c.phi, rho, u, cc, phi, type);
    return hipGetLastError();
}

hipError_t launch_fields(Ctx &c, double *rho, double *u, double *cc, double *phi, uint8_t *type) {
    if (c.Q == 9) return c.fp64 ? fields_impl<D2Q9, double>(c, rho, u, cc, phi, type) : fields_impl<D2Q9, float>(c, rho, u, cc, phi, type);
    return c.fp64 ? fields_impl<D3Q19, double>(c, rho, u, cc, phi, type) : fields_impl<D3Q19, float>(c, rho, u, cc, phi, type);
}

template <class L, typename T>
static hipError_t pops_impl(Ctx &c, double *f, double *g) {
    const long nb = (c.N + BLK - 1) / BLK;
    hipLaunchKernelGGL((k_pops<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.doms,
                       c.dnode_off, c.ndom, c.kof, (const T *)c.f[c.cur], (const T *)c.g[c.cur], f, g);
    return hipGetLastError();
}

hipError_t launch_pops(Ctx &c, double *f, double *g) {
    if (c.Q == 9) return c.fp64 ? pops_impl<D2Q9, double>(c, f, g) : pops_impl<D2Q9, float>(c, f, g);
    return c.fp64 ? pops_impl<D3Q19, double>(c, f, g) : pops_impl<D3Q19, float>(c, f, g);
}

template <typename T>
static hipError_t exchange_impl(Ctx &c, double *q) {
    const long nq = c.N * c.Q;
    hipLaunchKernelGGL(k_zero_f64, dim3((nq + BLK - 1) / BLK), dim3(BLK), 0, c.stream, q, nq);
    if (c.n_links > 0)
        hipLaunchKernelGGL((k_scatter_q<T>), dim3((c.n_links + BLK - 1) / BLK), dim3(BLK), 0,
                           c.stream, (long)c.n_links, c.Q, (const T *)c.lq, c.lnode, c.ldir, q);
    return hipGetLastError();
}

hipError_t launch_exchange(Ctx &c, double *q) {
    return c.fp64 ? exchange_impl<double>(c, q) : exchange_impl<float>(c, q);
}

template <class L, typename T>
static hipError_t diag_impl(Ctx &c, double *sums, int32_t *nan_flag) {
    const long nb = (c.N + BLK - 1) / BLK;
    hipError_t e = launch_fold_exchange(c);
    if (e == hipSuccess) e = launch_phi_flush(c);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, c.stream, c.iacc + 4);
    hipLaunchKernelGGL((k_diag<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.doms,
                       c.dnode_off, c.ndom, c.kof, (const T *)c.f[c.cur], (const T *)c.g[c.cur],
                       c.phi, c.dpart, c.iacc + 4);
    hipLaunchKernelGGL(k_sum_pairs, dim3(FOLD_G), dim3(BLK), 0, c.stream, (const double *)c.dpart, nb, c.fpart);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(BLK), 0, c.stream, (const double *)c.fpart, (long)FOLD_G,
                       c.dacc + 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(sums, c.dacc, 5 * sizeof(double), hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(nan_flag, c.iacc + 4, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c.stream);
}

hipError_t launch_diag(Ctx &c, double *sums, int32_t *nan_flag) {
    if (c.Q == 9) return c.fp64 ? diag_impl<D2Q9, double>(c, sums, nan_flag) : diag_impl<D2Q9, float>(c, sums, nan_flag);
    return c.fp64 ? diag_impl<D3Q19, double>(c, sums, nan_flag) : diag_impl<D3Q19, float>(c, sums, nan_flag);
}

}  // namespace lbm
