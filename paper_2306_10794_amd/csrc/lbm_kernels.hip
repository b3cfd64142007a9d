// lbm_kernels.hip -- gfx950 kernels of the reactive lattice Boltzmann step.
//
// Hot path per time step (both lattices in one pass over the nodes):
//   k_step       pull-stream with halfway bounce-back, moments, Guo-forced BGK
//                for the fluid; pull-stream, inlet/outlet planes, the reactive
//                boundary condition on every reactive link, advection-diffusion
//                BGK for the solute; writes the per-link exchange q and credits
//                precipitation (q < 0) to the fluid node's phi.
//   k_phi_solid  per solid interface node: dissolution (q > 0) charged to its
//                phi in link order, and the step's total wall exchange.
// Populations are stored structure-of-arrays, one contiguous array per
// direction with stride S (x fastest), ping-ponged between two buffers.  Each
// population value is read exactly once per step, so the kernel is a pure
// stream: no LDS staging is needed to avoid re-reads.
#include "lbm_internal.hpp"

namespace lbm {

constexpr int BLK = 256;

template <class L>
__device__ __forceinline__ long lin_off(int i, int nx, long nxy) {
    return (long)L::ex[i] + (long)L::ey[i] * nx + (long)L::ez[i] * nxy;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over a workgroup of BLK threads; result valid in thread 0
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[BLK / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BLK / 64; k++) s += part[k];
    return s;
}

// ---------------------------------------------------------------------------
// fused step
// ---------------------------------------------------------------------------
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_step(StepArgs<T> a, long nblocks) {
    // T: storage type of the populations; R: arithmetic type.  Arithmetic is
    // FP64 in both precisions: the step is bound by HBM traffic, and FP32
    // arithmetic on rounded weights would leak mass and momentum by a fixed
    // relative amount every collision.
    using R = double;
    constexpr int Q = L::Q;
    const long tile = xcd_tile(blockIdx.x, nblocks);
    const long n = tile * BLK + threadIdx.x;
    if (n >= a.N) return;
    const uint32_t fl = a.flags[n];
    if (!(fl & F_FLUID)) return;
    const long S = a.S;
    const int nx = a.box.nx;
    const long nxy = (long)nx * a.box.ny;
    const bool special = (fl & (F_FACE | F_DIRS)) != 0;
    const bool face = (fl & F_FACE) != 0;
    int X = 0, Y = 0, Z = 0;
    if (face) coords(a.box, n, &X, &Y, &Z);

    // ---- fluid: pull with halfway bounce-back ----
    R fp[Q];
    if (!special) {
#pragma unroll
        for (int i = 0; i < Q; i++) fp[i] = (R)a.fin[i * S + n - lin_off<L>(i, nx, nxy)];
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if (fl & (1u << i)) {
                fp[i] = (R)a.fin[L::opp[i] * S + n];
            } else {
                long y;
                if (face) {
                    int fc;
                    y = site(a.box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], false, &fc);
                } else {
                    y = n - lin_off<L>(i, nx, nxy);
                }
                fp[i] = (R)a.fin[i * S + y];
            }
        }
    }
    // moments (deviation form: sum_i w_i rho0 e_i = 0)
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        drho += fp[i];
        if (L::ex[i]) jx += L::ex[i] > 0 ? fp[i] : -fp[i];
        if (L::ey[i]) jy += L::ey[i] > 0 ? fp[i] : -fp[i];
        if (L::ez[i]) jz += L::ez[i] > 0 ? fp[i] : -fp[i];
    }
    const R rho = a.rho0 + drho;
    const R irho = R(1) / rho;
    // rho u = j + F/2 enters the first-order equilibrium term directly, so the
    // equilibrium carries exactly the momentum of the node
    const R mx = jx + R(0.5) * a.F[0], my = jy + R(0.5) * a.F[1], mz = jz + R(0.5) * a.F[2];
    const R ux = mx * irho, uy = my * irho, uz = mz * irho;
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * a.F[0] + uy * a.F[1] + uz * a.F[2];
    T *fo = a.fout;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
        const R em = R(L::ex[i]) * mx + R(L::ey[i]) * my + R(L::ez[i]) * mz;
        const R eF = R(L::ex[i]) * a.F[0] + R(L::ey[i]) * a.F[1] + R(L::ez[i]) * a.F[2];
        const R wi = R(L::w[i]);
        const R feq = wi * (drho + R(3) * em + rho * (R(4.5) * eu * eu - R(1.5) * uu));
        const R src = wi * (R(3) * (eF - uF) + R(9) * eu * eF);
        fo[i * S + n] = (T)(fp[i] + a.omega_f * (feq - fp[i]) + a.force_fac * src);
    }

    // ---- solute: pull, plane faces, reactive links ----
    R gp[Q];
    if (!special) {
#pragma unroll
        for (int i = 0; i < Q; i++) gp[i] = (R)a.gin[i * S + n - lin_off<L>(i, nx, nxy)];
    } else {
        const uint32_t rbc = (fl & F_LINK) ? a.rmask[n] : 0u;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            gp[i] = R(0);
            if (rbc & (1u << i)) continue;
            if (!face) {
                gp[i] = (R)a.gin[i * S + n - lin_off<L>(i, nx, nxy)];
                continue;
            }
            int fc;
            const long y = site(a.box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], true, &fc);
            if (y >= 0) {
                gp[i] = (R)a.gin[i * S + y];
            } else if (fc == 2 * a.box.inlet_axis) {
                const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
                gp[i] = a.ws[i] * (a.c_in - a.c_ref) + a.ws[i] * a.c_in * eu * a.inv_cs2s;
            } else if (fc == 2 * a.box.inlet_axis + 1) {
                const int ax = a.box.inlet_axis;
                int fc2;
                const long y2 = site(a.box, X, Y, Z, -L::ex[i] - (ax == 0), -L::ey[i] - (ax == 1),
                                     -L::ez[i] - (ax == 2), true, &fc2);
                if (y2 >= 0 && (a.flags[y2] & F_FLUID)) gp[i] = (R)a.gin[i * S + y2];
                else gp[i] = (R)a.gin[L::opp[i] * S + n];
            } else {
                gp[i] = (R)a.gin[L::opp[i] * S + n];
            }
        }
        if (rbc) {
            const int base = a.lbase[n];
            int r = 0;
            double sneg = 0.0;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if (rbc & (1u << i)) {
                    const int o = L::opp[i];
                    const R own = (R)a.gin[o * S + n];
                    const R beta = (R)a.lbeta[base + r];
                    const R src = (a.mech == LBM_PRECOLL && !(rbc & (1u << o))) ? gp[o] : own;
                    const R pin = (R(1) - beta) * (a.ws[i] * a.ceq_dev) + beta * src;
                    gp[i] = pin;
                    const T qv = (T)(pin - own);
                    a.lq[base + r] = qv;
                    if (qv < T(0)) sneg -= (double)qv;
                    r++;
                }
            }
            if (sneg != 0.0) a.phi[n] += a.vma * sneg;
        }
    }
    R dC = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) dC += gp[i];
    const R C = a.c_ref + dC;
    T *go = a.gout;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
        const R geq = a.ws[i] * (dC + C * eu * a.inv_cs2s);
        go[i * S + n] = (T)(gp[i] + a.omega_g * (geq - gp[i]));
    }
}

// dissolution side of the solid fraction, per solid interface node, links in
// ascending direction order; also the step's total exchange into acc[0]
template <typename T>
__global__ __launch_bounds__(BLK) void k_phi_solid(const int32_t *sif, const int32_t *soff,
                                                   const int32_t *slinks, const T *lq, double *phi,
                                                   long nsif, double vma, double *acc) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    double tot = 0.0;
    if (j < nsif) {
        const int s = sif[j];
        double pos = 0.0;
        const int k1 = soff[j + 1];
        for (int k = soff[j]; k < k1; k++) {
            const double qv = (double)lq[slinks[k]];
            tot += qv;
            if (qv > 0.0) pos += qv;
        }
        phi[s] -= vma * pos;
    }
    tot = block_sum(tot);
    if (threadIdx.x == 0 && tot != 0.0) atomicAdd(acc, tot);
}

template <typename T>
static StepArgs<T> step_args(Ctx &c) {
    StepArgs<T> a;
    a.fin = (const T *)c.f[c.cur];
    a.fout = (T *)c.f[1 - c.cur];
    a.gin = (const T *)c.g[c.cur];
    a.gout = (T *)c.g[1 - c.cur];
    a.flags = c.flags;
    a.rmask = c.rmask;
    a.lbase = c.lbase;
    a.lbeta = (const T *)c.lbeta;
    a.lq = (T *)c.lq;
    a.phi = c.phi;
    a.N = c.N;
    a.S = c.S;
    a.box = c.box;
    a.mech = c.p.rbc_mechanics;
    a.omega_f = 1.0 / c.p.tau_ns;
    a.omega_g = 1.0 / c.p.tau_ad;
    a.force_fac = 1.0 - 0.5 / c.p.tau_ns;
    for (int d = 0; d < 3; d++) a.F[d] = c.p.force[d];
    for (int i = 0; i < 19; i++) a.ws[i] = i < c.Q ? c.ws[i] : 0.0;
    a.inv_cs2s = 1.0 / c.cs2s;
    a.rho0 = c.fp64 ? 0.0 : c.p.rho0;
    a.c_ref = c.fp64 ? 0.0 : c.p.c_ref;
    a.ceq_dev = c.p.c_eq - (c.fp64 ? 0.0 : c.p.c_ref);
    a.c_in = c.p.inlet_axis >= 0 ? c.p.c_in : 0.0;
    a.vma = c.p.v_m * c.p.a_m;
    return a;
}

template <class L, typename T>
static hipError_t step_impl(Ctx &c, hipEvent_t *ev) {
    const long nb = (c.N + BLK - 1) / BLK;
    if (ev) (void)hipEventRecord(ev[0], c.stream);
    hipLaunchKernelGGL((k_step<L, T>), dim3(nb), dim3(BLK), 0, c.stream, step_args<T>(c), nb);
    hipError_t e = hipGetLastError();
    if (ev) (void)hipEventRecord(ev[1], c.stream);
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[2], c.stream);
    if (c.n_sif > 0) {
        const long nb2 = (c.n_sif + BLK - 1) / BLK;
        hipLaunchKernelGGL((k_phi_solid<T>), dim3(nb2), dim3(BLK), 0, c.stream, c.sif, c.soff,
                           c.slinks, (const T *)c.lq, c.phi, (long)c.n_sif, c.p.v_m * c.p.a_m,
                           c.dacc);
        e = hipGetLastError();
    }
    if (ev) (void)hipEventRecord(ev[3], c.stream);
    c.cur = 1 - c.cur;
    return e;
}

hipError_t launch_step(Ctx &c, hipEvent_t *ev) {
    if (c.Q == 9) return c.fp64 ? step_impl<D2Q9, double>(c, ev) : step_impl<D2Q9, float>(c, ev);
    return c.fp64 ? step_impl<D3Q19, double>(c, ev) : step_impl<D3Q19, float>(c, ev);
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (in place allowed); total written to *total
// ---------------------------------------------------------------------------
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = BLK * SCAN_PER;

__global__ __launch_bounds__(BLK) void k_scan_reduce(const int32_t *in, long n, int32_t *bsum) {
    const long base = (long)blockIdx.x * SCAN_TILE;
    long s = 0;
    for (int k = 0; k < SCAN_PER; k++) {
        const long i = base + (long)k * BLK + threadIdx.x;
        if (i < n) s += in[i];
    }
    const double t = block_sum((double)s);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int32_t)t;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *bsum, long nb, int32_t *total) {
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long c0 = 0; c0 < nb; c0 += 1024) {
        const long i = c0 + threadIdx.x;
        const int32_t v = i < nb ? bsum[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(BLK) void k_scan_down(const int32_t *in, int32_t *out, long n,
                                                   const int32_t *bsum) {
    __shared__ int32_t tsum[BLK];
    const long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        const long i = base + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    tsum[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < BLK; off <<= 1) {
        const int32_t add = threadIdx.x >= off ? tsum[threadIdx.x - off] : 0;
        __syncthreads();
        tsum[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = bsum[blockIdx.x] + tsum[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        const long i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

static hipError_t scan_excl(Ctx &c, const int32_t *in, int32_t *out, long n, int32_t *total_dev) {
    const long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(BLK), 0, c.stream, in, n, c.bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, c.stream, c.bsum, nb, total_dev);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(BLK), 0, c.stream, in, out, n, c.bsum);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// geometry prep
// ---------------------------------------------------------------------------
template <class L>
__global__ __launch_bounds__(BLK) void k_flags(Box box, long N, const uint8_t *solid,
                                               uint32_t *flags, uint32_t *rmask, int32_t *cnt) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        flags[n] = 0u;
        rmask[n] = 0u;
        cnt[n] = 0;
        return;
    }
    int X, Y, Z;
    coords(box, n, &X, &Y, &Z);
    uint32_t fl = F_FLUID, rm = 0u;
    const bool face = X == 0 || X == box.nx - 1 || Y == 0 || Y == box.ny - 1 ||
                      (L::DIM == 3 && (Z == 0 || Z == box.nz - 1));
    if (face) fl |= F_FACE;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        int fc;
        const long y = site(box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], false, &fc);
        if (y < 0 || solid[y]) fl |= 1u << i;
        const long ys = site(box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], true, &fc);
        if (ys >= 0 && solid[ys]) rm |= 1u << i;
    }
    if (rm) fl |= F_LINK;
    flags[n] = fl;
    rmask[n] = rm;
    cnt[n] = __popc(rm);
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_links(Box box, long N, const uint32_t *flags,
                                               const uint32_t *rmask, const int32_t *lbase,
                                               const double *nrm, const double *kr, int scheme,
                                               int mech, double gamma, double cs2s, T *lbeta,
                                               int32_t *lnode, int32_t *lsolid, uint8_t *ldir) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (!(flags[n] & F_LINK)) return;
    int X, Y, Z;
    coords(box, n, &X, &Y, &Z);
    const uint32_t rm = rmask[n];
    const int base = lbase[n];
    int r = 0;
    for (int i = 1; i < L::Q; i++) {
        if (!(rm & (1u << i))) continue;
        int fc;
        const long s = site(box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], true, &fc);
        const double en = L::ex[i] * nrm[3 * s] + L::ey[i] * nrm[3 * s + 1] + L::ez[i] * nrm[3 * s + 2];
        const double k = kr[s];
        double kap;
        if (scheme == LBM_SV) kap = en > 0 ? k * en / cs2s : 0.0;
        else if (scheme == LBM_SPJ) kap = en > 0 ? gamma * k / (cs2s * en) : 0.0;
        else kap = en > 0 ? gamma * k * en / cs2s : 0.0;
        // pre-collision source with both neighbours solid: fall back to the
        // node's own post-collision population, whose effective rate is gamma k
        if (mech == LBM_PRECOLL && (rm & (1u << L::opp[i]))) kap = kap / gamma;
        const double beta = scheme == LBM_ABB ? -1.0 : (1.0 - kap) / (1.0 + kap);
        lbeta[base + r] = (T)beta;
        lnode[base + r] = (int32_t)n;
        lsolid[base + r] = (int32_t)s;
        ldir[base + r] = (uint8_t)i;
        r++;
    }
}

template <class L>
__device__ __forceinline__ int solid_links(const Box &box, long n, const uint8_t *solid,
                                           const uint32_t *rmask, const int32_t *lbase,
                                           int32_t *out) {
    int X, Y, Z;
    coords(box, n, &X, &Y, &Z);
    int k = 0;
    for (int i = 1; i < L::Q; i++) {
        int fc;
        const long x = site(box, X, Y, Z, L::ex[i], L::ey[i], L::ez[i], true, &fc);
        if (x < 0 || solid[x]) continue;
        const uint32_t rm = rmask[x];
        if (!(rm & (1u << i))) continue;
        if (out) out[k] = lbase[x] + __popc(rm & ((1u << i) - 1u));
        k++;
    }
    return k;
}

template <class L>
__global__ __launch_bounds__(BLK) void k_solid_count(Box box, long N, const uint8_t *solid,
                                                     const uint32_t *rmask, int32_t *cnt,
                                                     int32_t *ind) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    int k = 0;
    if (solid[n]) k = solid_links<L>(box, n, solid, rmask, nullptr, nullptr);
    cnt[n] = k;
    ind[n] = k > 0 ? 1 : 0;
}

template <class L>
__global__ __launch_bounds__(BLK) void k_solid_fill(Box box, long N, const uint8_t *solid,
                                                    const uint32_t *rmask, const int32_t *lbase,
                                                    const int32_t *off, const int32_t *idx,
                                                    int32_t *sif, int32_t *soff, int32_t *slinks) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (!solid[n]) return;
    const int k = solid_links<L>(box, n, solid, rmask, lbase, slinks + off[n]);
    if (k > 0) {
        sif[idx[n]] = (int32_t)n;
        soff[idx[n]] = off[n];
    }
}

// lattice-gradient normal of the solid indicator (used when no normals are given)
template <class L>
__global__ __launch_bounds__(BLK) void k_fd_normals(Box box, long N, const uint8_t *solid,
                                                    double *nrm) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    double gx = 0, gy = 0, gz = 0;
    if (solid[n]) {
        int X, Y, Z;
        coords(box, n, &X, &Y, &Z);
        for (int i = 1; i < L::Q; i++) {
            int fc;
            const long y = site(box, X, Y, Z, L::ex[i], L::ey[i], L::ez[i], false, &fc);
            const double ind = (y < 0 || solid[y]) ? 1.0 : 0.0;
            gx += L::w[i] * L::ex[i] * ind * 3.0;
            gy += L::w[i] * L::ey[i] * ind * 3.0;
            gz += L::w[i] * L::ez[i] * ind * 3.0;
        }
        const double m = sqrt(gx * gx + gy * gy + gz * gz);
        if (m > 0) { gx = -gx / m; gy = -gy / m; gz = -gz / m; }
        else { gx = gy = gz = 0.0; }
    }
    nrm[3 * n] = gx;
    nrm[3 * n + 1] = gy;
    nrm[3 * n + 2] = gz;
}

__global__ __launch_bounds__(BLK) void k_node_defaults(long N, const uint8_t *solid, const double *kr_in,
                                                       double kr0, const double *phi_in, double *kr,
                                                       double *phi) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    kr[n] = kr_in ? kr_in[n] : kr0;
    phi[n] = phi_in ? phi_in[n] : (solid[n] ? 1.0 : 0.0);
}

__global__ __launch_bounds__(BLK) void k_copy_solid(long N, const uint8_t *in, uint8_t *out) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    out[n] = in[n] ? 1 : 0;
}

__global__ void k_set_last(int32_t *soff, long nsif, int32_t v) { soff[nsif] = v; }

__global__ void k_zero_i32(int32_t *p, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// fluid nodes and fluid interface nodes, into cnt[0], cnt[1]
__global__ __launch_bounds__(BLK) void k_count_nodes(long N, const uint32_t *flags, int32_t *cnt) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (n < N) {
        const uint32_t fl = flags[n];
        a = (fl & F_FLUID) ? 1.0 : 0.0;
        b = (fl & F_LINK) ? 1.0 : 0.0;
    }
    a = block_sum(a);
    __syncthreads();
    b = block_sum(b);
    if (threadIdx.x == 0) {
        atomicAdd(cnt, (int32_t)a);
        atomicAdd(cnt + 1, (int32_t)b);
    }
}

template <class L, typename T>
static hipError_t geometry_impl(Ctx &c, const uint8_t *solid, const double *normals,
                                const double *k_r, const double *phi0, int64_t *n_links,
                                int64_t *n_sif) {
    const long N = c.N;
    const long nb = (N + BLK - 1) / BLK;
    hipStream_t st = c.stream;
    hipLaunchKernelGGL(k_copy_solid, dim3(nb), dim3(BLK), 0, st, N, solid, c.solid);
    hipLaunchKernelGGL(k_node_defaults, dim3(nb), dim3(BLK), 0, st, N, c.solid, k_r, c.p.k_r,
                       phi0, c.kr, c.phi);
    if (normals) {
        hipError_t e = hipMemcpyAsync(c.nrm, normals, sizeof(double) * 3 * N,
                                      hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL((k_fd_normals<L>), dim3(nb), dim3(BLK), 0, st, c.box, N, c.solid, c.nrm);
    }
    hipLaunchKernelGGL((k_flags<L>), dim3(nb), dim3(BLK), 0, st, c.box, N, c.solid, c.flags,
                       c.rmask, c.cnt);
    hipError_t e = scan_excl(c, c.cnt, c.lbase, N, c.iacc);
    if (e != hipSuccess) return e;
    int32_t tot = 0;
    e = hipMemcpyAsync(&tot, c.iacc, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *n_links = tot;
    if (tot > c.max_links) return hipSuccess;  // caller reports the capacity error
    hipLaunchKernelGGL((k_links<L, T>), dim3(nb), dim3(BLK), 0, st, c.box, N, c.flags, c.rmask,
                       c.lbase, c.nrm, c.kr, c.p.rbc_scheme, c.p.rbc_mechanics, c.gamma, c.cs2s,
                       (T *)c.lbeta, c.lnode, c.lsolid, c.ldir);
    hipLaunchKernelGGL((k_solid_count<L>), dim3(nb), dim3(BLK), 0, st, c.box, N, c.solid, c.rmask,
                       c.cnt, c.sidx);
    e = scan_excl(c, c.sidx, c.sidx, N, c.iacc);
    if (e != hipSuccess) return e;
    e = scan_excl(c, c.cnt, c.cnt, N, c.iacc + 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, c.iacc + 2, 2);
    hipLaunchKernelGGL(k_count_nodes, dim3(nb), dim3(BLK), 0, st, N, c.flags, c.iacc + 2);
    int32_t t2[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(t2, c.iacc, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *n_sif = t2[0];
    c.n_fluid = t2[2];
    c.n_fluid_iface = t2[3];
    hipLaunchKernelGGL((k_solid_fill<L>), dim3(nb), dim3(BLK), 0, st, c.box, N, c.solid, c.rmask,
                       c.lbase, c.cnt, c.sidx, c.sif, c.soff, c.slinks);
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, c.soff, (long)t2[0], t2[1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t2[1] != tot) return hipErrorUnknown;  // every link must have one solid end
    return hipStreamSynchronize(st);
}

hipError_t launch_geometry(Ctx &c, const uint8_t *solid, const double *normals, const double *k_r,
                           const double *phi0, int64_t *n_links, int64_t *n_sif) {
    if (c.Q == 9)
        return c.fp64 ? geometry_impl<D2Q9, double>(c, solid, normals, k_r, phi0, n_links, n_sif)
                      : geometry_impl<D2Q9, float>(c, solid, normals, k_r, phi0, n_links, n_sif);
    return c.fp64 ? geometry_impl<D3Q19, double>(c, solid, normals, k_r, phi0, n_links, n_sif)
                  : geometry_impl<D3Q19, float>(c, solid, normals, k_r, phi0, n_links, n_sif);
}

// ---------------------------------------------------------------------------
// initial state and read-outs
// ---------------------------------------------------------------------------
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_init(long N, long S, const uint8_t *solid, const double *rho,
                                              const double *u, const double *cc, double rho0,
                                              double c_ref, const double *ws, double cs2s, T *f0,
                                              T *g0, T *f1, T *g1) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        for (int i = 0; i < L::Q; i++) {
            f0[i * S + n] = T(0); g0[i * S + n] = T(0);
            f1[i * S + n] = T(0); g1[i * S + n] = T(0);
        }
        return;
    }
    const double r = rho ? rho[n] : 1.0;
    const double ux = u ? u[3 * n] : 0.0, uy = u ? u[3 * n + 1] : 0.0, uz = u ? u[3 * n + 2] : 0.0;
    const double C = cc ? cc[n] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < L::Q; i++) {
        const double eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
        const double feq = L::w[i] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        const double geq = ws[i] * C * (1.0 + eu / cs2s);
        f0[i * S + n] = T(feq - L::w[i] * rho0);
        g0[i * S + n] = T(geq - ws[i] * c_ref);
        f1[i * S + n] = T(0);
        g1[i * S + n] = T(0);
    }
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_fields(long N, long S, const uint8_t *solid, const T *f,
                                                const T *g, double rho0, double c_ref,
                                                const double *F, const double *phi_in,
                                                double *rho, double *u, double *cc, double *phi,
                                                uint8_t *type) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    double r = 0, jx = 0, jy = 0, jz = 0, C = 0;
    const bool sol = solid[n] != 0;
    if (!sol) {
        double dr = 0, dc = 0;
        for (int i = 0; i < L::Q; i++) {
            const double fi = (double)f[i * S + n];
            dr += fi;
            jx += L::ex[i] * fi;
            jy += L::ey[i] * fi;
            jz += L::ez[i] * fi;
            dc += (double)g[i * S + n];
        }
        r = rho0 + dr;
        C = c_ref + dc;
    }
    if (rho) rho[n] = r;
    if (u) {
        u[3 * n] = sol ? 0.0 : (jx - 0.5 * F[0]) / r;
        u[3 * n + 1] = sol ? 0.0 : (jy - 0.5 * F[1]) / r;
        u[3 * n + 2] = sol ? 0.0 : (jz - 0.5 * F[2]) / r;
    }
    if (cc) cc[n] = C;
    if (phi) phi[n] = phi_in[n];
    if (type) type[n] = sol ? 1 : 0;
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_pops(long N, long S, const uint8_t *solid, const T *f,
                                              const T *g, double rho0, double c_ref,
                                              const double *ws, double *fo, double *go) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    const bool sol = solid[n] != 0;
    for (int i = 0; i < L::Q; i++) {
        if (fo) fo[i * N + n] = sol ? 0.0 : (double)f[i * S + n] + L::w[i] * rho0;
        if (go) go[i * N + n] = sol ? 0.0 : (double)g[i * S + n] + ws[i] * c_ref;
    }
}

__global__ __launch_bounds__(BLK) void k_zero_f64(double *p, long n) {
    const long i = (long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_scatter_q(long nl, int Q, const T *lq, const int32_t *lnode,
                                                   const uint8_t *ldir, double *q) {
    const long k = (long)blockIdx.x * BLK + threadIdx.x;
    if (k < nl) q[(long)lnode[k] * Q + ldir[k]] = (double)lq[k];
}

template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_diag(long N, long S, const uint8_t *solid, const T *f,
                                              const T *g, const double *phi, double c_ref,
                                              double *acc, int32_t *nan_flag) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    double cs = 0.0, ps = 0.0;
    int bad = 0;
    if (n < N) {
        ps = phi[n];
        if (!solid[n]) {
            double dc = 0.0;
            for (int i = 0; i < L::Q; i++) {
                const double fi = (double)f[i * S + n], gi = (double)g[i * S + n];
                if (!isfinite(fi) || !isfinite(gi)) bad = 1;
                dc += gi;
            }
            cs = c_ref + dc;
        }
    }
    const double bc = block_sum(cs);
    __syncthreads();
    const double bp = block_sum(ps);
    if (threadIdx.x == 0) {
        atomicAdd(acc, bc);
        atomicAdd(acc + 1, bp);
    }
    if (bad) atomicOr(nan_flag, 1);
}

template <class L, typename T>
static hipError_t init_impl(Ctx &c, const double *rho, const double *u, const double *cc) {
    const long nb = (c.N + BLK - 1) / BLK;
    double *wsd = c.dacc + 8;  // solute weights staged in the accumulator block
    hipError_t e = hipMemcpyAsync(wsd, c.ws, sizeof(double) * 19, hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return e;
    c.cur = 0;
    hipLaunchKernelGGL((k_init<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.solid, rho, u,
                       cc, c.fp64 ? 0.0 : c.p.rho0, c.fp64 ? 0.0 : c.p.c_ref, wsd, c.cs2s,
                       (T *)c.f[0], (T *)c.g[0], (T *)c.f[1], (T *)c.g[1]);
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(BLK), 0, c.stream, c.dacc, 8);
    return hipGetLastError();
}

hipError_t launch_init(Ctx &c, const double *rho, const double *u, const double *cc) {
    if (c.Q == 9) return c.fp64 ? init_impl<D2Q9, double>(c, rho, u, cc) : init_impl<D2Q9, float>(c, rho, u, cc);
    return c.fp64 ? init_impl<D3Q19, double>(c, rho, u, cc) : init_impl<D3Q19, float>(c, rho, u, cc);
}

template <class L, typename T>
static hipError_t fields_impl(Ctx &c, double *rho, double *u, double *cc, double *phi, uint8_t *type) {
    const long nb = (c.N + BLK - 1) / BLK;
    double *Fd = c.dacc + 28;
    hipError_t e = hipMemcpyAsync(Fd, c.p.force, sizeof(double) * 3, hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fields<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.solid,
                       (const T *)c.f[c.cur], (const T *)c.g[c.cur], c.fp64 ? 0.0 : c.p.rho0,
                       c.fp64 ? 0.0 : c.p.c_ref, Fd, c.phi, rho, u, cc, phi, type);
    return hipGetLastError();
}

hipError_t launch_fields(Ctx &c, double *rho, double *u, double *cc, double *phi, uint8_t *type) {
    if (c.Q == 9) return c.fp64 ? fields_impl<D2Q9, double>(c, rho, u, cc, phi, type) : fields_impl<D2Q9, float>(c, rho, u, cc, phi, type);
    return c.fp64 ? fields_impl<D3Q19, double>(c, rho, u, cc, phi, type) : fields_impl<D3Q19, float>(c, rho, u, cc, phi, type);
}

template <class L, typename T>
static hipError_t pops_impl(Ctx &c, double *f, double *g) {
    const long nb = (c.N + BLK - 1) / BLK;
    double *wsd = c.dacc + 8;
    hipError_t e = hipMemcpyAsync(wsd, c.ws, sizeof(double) * 19, hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pops<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.solid,
                       (const T *)c.f[c.cur], (const T *)c.g[c.cur], c.fp64 ? 0.0 : c.p.rho0,
                       c.fp64 ? 0.0 : c.p.c_ref, wsd, f, g);
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
    double *acc = c.dacc + 1;
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(BLK), 0, c.stream, acc, 2);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c.stream, c.iacc + 4, 1);
    hipError_t e;
    hipLaunchKernelGGL((k_diag<L, T>), dim3(nb), dim3(BLK), 0, c.stream, c.N, c.S, c.solid,
                       (const T *)c.f[c.cur], (const T *)c.g[c.cur], c.phi,
                       c.fp64 ? 0.0 : c.p.c_ref, acc, c.iacc + 4);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(sums, c.dacc, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream);
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
