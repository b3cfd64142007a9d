// lbm_adjoint.hip -- gradient of a loss on the final concentrations with
// respect to the rate constants k_r of the solid nodes.
//
// The fluid does not depend on k_r; the adjoint covers a fluid at rest
// (u = 0: pure reaction-diffusion), so only the solute lattice is
// differentiated.  A recorded forward run keeps the solute state every
// `ckpt` steps.  The backward pass walks the segments from the last: it
// recomputes the segment's states from its checkpoint (solute-only step,
// k_sol_step) and then applies the transposed step (k_adj_step) from the last
// state of the segment to its first.
//
// Transposed step.  lambda(t) = dL/dg*(t), the adjoint of the post-collision
// populations.  Forward, at a fluid node x: p_i = g*_i(x - e_i) (pull), or
// g*_o(x) with o = opp(i) (bounce-back at a box face), or on a reactive link
// (x - e_i solid) p_i = (1 - beta_i) w_i C_eq + beta_i src_i with src_i the
// pulled p_o (pre-collision mechanics, when o is not reactive) or the own
// g*_o(x); then g*_i = (1 - w) p_i + w w_i C (C = sum p).  The transpose of
// the collision is nu_j = (1 - w) mu_j + w sum_i w_i mu_i with mu = lambda(t+1)
// at x; the rate condition passes beta_i nu_i on to its source; the pull is
// transposed into a pull in the opposite direction.  Every node writes, per
// direction j, one value into an array P laid out like the populations:
//   kk[j] >= 0 or a box face: nu_j plus what reactive links passed to p_j,
//                             read by the node that p_j was pulled from;
//   a reactive link:          beta_j nu_j if its source is the node's own
//                             g*_o (else 0), the node's own lambda_o.
// so that lambda_d(x, t) = P[d][kk[opp d]] if x + e_d is fluid, else
// P[opp d][x]: the same gather as the forward pull, directions reversed.
// dL/dbeta of each link accumulates nu_i (src_i - w_i C_eq) over the steps:
// each transposed step writes its term over the link's source value (storage
// precision), and after a segment one kernel adds the segment's terms to the
// FP64 total, one lane per link, in the order the steps ran; a last kernel
// turns it into dL/dk_r per solid node through dbeta/dk_r of the link's
// scheme, summing its links in direction order.
#include "lbm_internal.hpp"
#include "lbm_task.hpp"

namespace lbm {

template <typename T>
struct AdjArgs {
    const T *__restrict__ pin;    // adjoint array of step t+1 (P layout)
    T *__restrict__ pout;         // adjoint array of step t
    const T *__restrict__ gin;    // solute state the forward step started from
    T *__restrict__ gout;         // solute state after the step (recompute)
    const Task *__restrict__ tasks;
    const RowWord *__restrict__ rows;
    const DomDev *__restrict__ doms;
    const int32_t *__restrict__ nodeof;
    const int32_t *__restrict__ lbase;
    const T *__restrict__ lbeta;
    T *__restrict__ lsrc;         // per link: the source value of its rate condition
                                  // (written by the recomputation, read by the transpose)
    double *__restrict__ gbeta;   // per link dL/dbeta, accumulated
    const double *__restrict__ dldc;  // dense dL/dC_T (init)
    long ntasks, S;
};

// A task's per-link values staged in LDS as 32-bit words (word w of element
// j at [w][j]): fetched straight from global memory into LDS, so that no
// register waits on them and the population loads issue behind them at once.
template <typename V, int CAP>
__device__ __forceinline__ void lds_fetch(const V *__restrict__ src, uint32_t (&dst)[sizeof(V) / 4][CAP], int n,
                                          int lane) {
    for (int c = 0; c < n; c += 64)
        if (c + lane < n) {
            const uint32_t *p = (const uint32_t *)(src + c + lane);
#pragma unroll
            for (int w = 0; w < (int)(sizeof(V) / 4); w++)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(p + w),
                                                 (__attribute__((address_space(3))) void *)&dst[w][c], 4, 0, 0);
        }
}

template <typename V, int CAP>
__device__ __forceinline__ V lds_get(const uint32_t (&src)[sizeof(V) / 4][CAP], int j) {
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, src[0][j]);
    } else {
        return __builtin_bit_cast(V, (unsigned long long)src[0][j] | ((unsigned long long)src[1][j] << 32));
    }
}

template <typename V, int CAP>
__device__ __forceinline__ void lds_put(uint32_t (&dst)[sizeof(V) / 4][CAP], int j, V v) {
    if constexpr (sizeof(V) == 4) {
        dst[0][j] = __builtin_bit_cast(uint32_t, v);
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        dst[0][j] = (uint32_t)b;
        dst[1][j] = (uint32_t)(b >> 32);
    }
}

// per-wavefront task setup shared by the three kernels; returns false for a
// wavefront without a task
template <class L, typename T>
struct TaskCtx {
    DomDev D;
    int kk[L::Q];
    uint32_t solidnb, cross, cross_hi;
    int k, n, lb;
    bool active;
};

template <class L, typename T>
__device__ __forceinline__ bool task_setup(const AdjArgs<T> &a, TaskCtx<L, T> &c) {
    // consecutive workgroups of tasks on one XCD (its L2 then holds the lines
    // that neighbouring tasks' pulls share), as in the fused step
    const long tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = __builtin_amdgcn_readfirstlane((int)(tile * (BLK / 64)) + (int)(threadIdx.x >> 6));
    if (t >= a.ntasks) return false;
    const int lane = threadIdx.x & 63;
    const Task tk = a.tasks[t];
    c.D = a.doms[tk.dom];
    const Box b = c.D.box;
    const int W = c.D.W;
    const RowWord *__restrict__ rows = a.rows + c.D.word_off;
    const int y0 = tk.y0, z = tk.z;
    const int cnt = tk.cnt & 255, nr = tk.cnt >> 8;
    const RowSlots rs = load_row_slots<L>(rows, b, W, lane, y0, z, nr, tk.wlo, tk.nwd);
    c.active = lane < cnt;
    c.k = tk.k0 + (c.active ? lane : 0);
    const int ry = task_row<L>(rs, W, nr, c.k);
    c.n = a.nodeof[c.k];
    c.lb = a.lbase[c.k];
    const int x = (int)(c.n - c.D.node_off) - (tk.row + ry) * b.nx;
    classify<L>(rows, b, W, rs, ry, x, y0 + ry, z, c.k, c.kk, c.solidnb, c.cross, c.cross_hi);
    return true;
}

// One solute step with the fluid at rest, from gin to gout: the arithmetic of
// the fused step's solute half with u = 0 (no exchange or solid fraction is
// written).  Each reactive link's source value goes to lsrc; with gout null
// only those are written.
template <class L, typename T, bool RED, bool TRT>
__global__ __launch_bounds__(BLK) void k_sol_step(AdjArgs<T> a) {
    using R = double;
    constexpr int Q = L::Q;
    constexpr uint32_t SM = sol_mask<L, RED>();   // the solute set (D2Q5 / D3Q7 when RED)
    constexpr int QS = __builtin_popcount(SM);
    constexpr int LCAP = 256;   // links of a task staged in LDS (more: read in place)
    constexpr int NW = (int)(sizeof(T) / 4);
    __shared__ uint32_t sb[BLK / 64][NW][LCAP], ss[BLK / 64][NW][LCAP];
    TaskCtx<L, T> c;
    if (!task_setup<L, T>(a, c)) return;
    const bool act = c.active;
    const DomDev &D = c.D;
    const long S = a.S;
    const uint32_t rbc = act ? (c.solidnb & SM) : 0u;
    // link index: the task's base (lbase of its first node, lane 0, which is
    // active), then by direction, then by lane
    const int lt = __builtin_amdgcn_readfirstlane(c.lb);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    int lpos[Q];
    int nlt = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (!((SM >> i) & 1u)) continue;
        const unsigned long long bal = __ballot((rbc >> i) & 1u);
        lpos[i] = nlt + __popcll(bal & below);
        nlt += __popcll(bal);
    }
    const bool staged = nlt <= LCAP;
    if (staged) lds_fetch<T, LCAP>(a.lbeta + lt, sb[wv], nlt, lane);
    const long ob = blk0(c.k, QS);
    T gv[Q];
    if (act) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if (!((SM >> i) & 1u)) continue;
            gv[i] = a.gin[c.kk[i] >= 0 ? pidx(sol_slot(SM, i), c.kk[i], QS) : ob + 64 * sol_slot(SM, L::opp[i])];
        }
    }
    // the coefficients in LDS, on every path (the loads above are needed now too)
    if (staged) lds_dma_wait();
    if (act) {
        // a pulled source is a direction without a link, which this loop
        // leaves unchanged
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (!((SM >> i) & 1u) || !(rbc & (1u << i))) continue;
            const int o = L::opp[i];
            const int pos = lpos[i];
            const R own = (R)gv[i];
            const R srcv = (D.mech == LBM_PRECOLL && !(rbc & (1u << o))) ? (R)gv[o] : own;
            const R beta = (R)(staged ? lds_get<T, LCAP>(sb[wv], pos) : a.lbeta[lt + pos]);
            if (staged) lds_put<T, LCAP>(ss[wv], pos, (T)srcv);
            else a.lsrc[lt + pos] = (T)srcv;
            gv[i] = (T)((R(1) - beta) * (sol_w<L>(D, i) * D.ceq_dev) + beta * srcv);
        }
        if (a.gout) {
            R dC = R(0);
#pragma unroll
            for (int i = 0; i < Q; i++)
                if ((SM >> i) & 1u) dC += (R)gv[i];
            if constexpr (TRT) {
                // TRT at rest: even parts relax with omega_gs toward w C, odd
                // parts with omega_g toward 0 (as the fused step with u = 0)
                const R oms = D.omega_gs, oma = D.omega_g;
                a.gout[ob] = (T)((R(1) - oms) * (R)gv[0] + oms * sol_w<L>(D, 0) * dC);
#pragma unroll
                for (int i = 1; i < Q; i++) {
                    if (L::opp[i] < i || !((SM >> i) & 1u)) continue;
                    const int o = L::opp[i];
                    const R gi = (R)gv[i], go = (R)gv[o];
                    const R As = oms * sol_w<L>(D, i) * dC;
                    const R hs = R(0.5) * oms * (gi + go), ha = R(0.5) * oma * (gi - go);
                    a.gout[ob + 64 * sol_slot(SM, i)] = (T)(gi - hs - ha + As);
                    a.gout[ob + 64 * sol_slot(SM, o)] = (T)(go - hs + ha + As);
                }
            } else {
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    if (!((SM >> i) & 1u)) continue;
                    const R gi = (R)gv[i];
                    const R geq = sol_w<L>(D, i) * dC;
                    a.gout[ob + 64 * sol_slot(SM, i)] = (T)(gi + D.omega_g * (geq - gi));
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (staged) {
#pragma unroll
        for (int r = 0; r < LCAP / 64; r++)
            if (r * 64 + lane < nlt) a.lsrc[lt + r * 64 + lane] = lds_get<T, LCAP>(ss[wv], r * 64 + lane);
    }
}

// lambda(T)_i(x) = dL/dC_T(x) for every i, written in the P layout
template <class L, typename T, bool RED>
__global__ __launch_bounds__(BLK) void k_adj_init(AdjArgs<T> a) {
    constexpr int Q = L::Q;
    constexpr uint32_t SM = sol_mask<L, RED>();
    constexpr int QS = __builtin_popcount(SM);
    TaskCtx<L, T> c;
    if (!task_setup<L, T>(a, c) || !c.active) return;
    const long S = a.S;
    const double own = a.dldc[c.n];
#pragma unroll
    for (int j = 0; j < Q; j++)
        if ((SM >> j) & 1u)
            a.pout[pidx(sol_slot(SM, j), c.k, QS)] = (T)(c.kk[j] >= 0 ? a.dldc[a.nodeof[c.kk[j]]] : own);
}

template <class L, typename T, bool RED, bool TRT>
__global__ __launch_bounds__(BLK) void k_adj_step(AdjArgs<T> a) {
    using R = double;
    constexpr int Q = L::Q;
    constexpr uint32_t SM = sol_mask<L, RED>();
    constexpr int QS = __builtin_popcount(SM);
    constexpr int LCAP = 256;   // links of a task staged in LDS (more: read in place)
    constexpr int NW = (int)(sizeof(T) / 4);
    __shared__ uint32_t sb[BLK / 64][NW][LCAP], ss[BLK / 64][NW][LCAP];
    TaskCtx<L, T> c;
    if (!task_setup<L, T>(a, c)) return;
    const bool act = c.active;
    const DomDev &D = c.D;
    const long S = a.S;
    const uint32_t rbc = act ? (c.solidnb & SM) : 0u;
    const int lt = __builtin_amdgcn_readfirstlane(c.lb);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    int lpos[Q];
    int nlt = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (!((SM >> i) & 1u)) continue;
        const unsigned long long bal = __ballot((rbc >> i) & 1u);
        lpos[i] = nlt + __popcll(bal & below);
        nlt += __popcll(bal);
    }
    const bool staged = nlt <= LCAP;
    if (staged) {
        lds_fetch<T, LCAP>(a.lbeta + lt, sb[wv], nlt, lane);
        lds_fetch<T, LCAP>(a.lsrc + lt, ss[wv], nlt, lane);
    }
    const long ob = blk0(c.k, QS);
    // lambda(t+1) at this node: the forward pull with directions reversed
    T mu[Q];
    if (act) {
#pragma unroll
        for (int d = 0; d < Q; d++) {
            if (!((SM >> d) & 1u)) continue;
            const int kd = c.kk[L::opp[d]];
            mu[d] = a.pin[kd >= 0 ? pidx(sol_slot(SM, d), kd, QS) : ob + 64 * sol_slot(SM, L::opp[d])];
        }
    }
    // the link values in LDS, on every path (the loads above are needed now too)
    if (staged) lds_dma_wait();
    if (act) {
        R m = R(0);
#pragma unroll
        for (int i = 0; i < Q; i++)
            if ((SM >> i) & 1u) m += sol_w<L>(D, i) * (R)mu[i];
        const R om = D.omega_g, om1 = R(1) - om, oms = D.omega_gs;
        const R ta = R(1) - R(0.5) * (oms + om), tb = R(0.5) * (om - oms);
        a.pout[ob] = (T)(TRT ? (R(1) - oms) * (R)mu[0] + oms * m : om1 * (R)mu[0] + om * m);
        auto link = [&](int d, R nu, R *out_d, R *out_other, bool pulled) {
            const int pos = lpos[d];
            const R beta = (R)(staged ? lds_get<T, LCAP>(sb[wv], pos) : a.lbeta[lt + pos]);
            const R src = (R)(staged ? lds_get<T, LCAP>(ss[wv], pos) : a.lsrc[lt + pos]);
            // this step's term of dL/dbeta replaces the source value (read
            // once, just above); the segment's terms are summed by k_adj_fold
            const T add = (T)(nu * (src - sol_w<L>(D, d) * D.ceq_dev));
            if (staged) lds_put<T, LCAP>(ss[wv], pos, add);
            else a.lsrc[lt + pos] = add;
            if (pulled) {
                *out_other += beta * nu;
                *out_d = R(0);
            } else {
                *out_d = beta * nu;
            }
        };
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (L::opp[i] < i || !((SM >> i) & 1u)) continue;
            const int o = L::opp[i];
            const int si = sol_slot(SM, i), so = sol_slot(SM, o);
            R nui, nuo;
            if constexpr (TRT) {
                nui = ta * (R)mu[i] + tb * (R)mu[o] + oms * m;
                nuo = ta * (R)mu[o] + tb * (R)mu[i] + oms * m;
            } else {
                nui = om1 * (R)mu[i] + om * m;
                nuo = om1 * (R)mu[o] + om * m;
            }
            R outi = nui, outo = nuo;
            const bool li = (rbc >> i) & 1u, lo = (rbc >> o) & 1u;
            if (li) link(i, nui, &outi, &outo, D.mech == LBM_PRECOLL && !lo);
            if (lo) link(o, nuo, &outo, &outi, D.mech == LBM_PRECOLL && !li);
            a.pout[ob + 64 * si] = (T)outi;
            a.pout[ob + 64 * so] = (T)outo;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (staged) {
#pragma unroll
        for (int r = 0; r < LCAP / 64; r++) {
            const int j = r * 64 + lane;
            if (j < nlt) a.lsrc[lt + j] = lds_get<T, LCAP>(ss[wv], j);
        }
    }
}

// dL/dbeta of every link += the terms its segment's transposed steps wrote
// over the source values, in the order those steps ran (last step first), in
// FP64: the same sums as adding each step's term as it is formed.
template <typename T>
__global__ __launch_bounds__(BLK) void k_adj_fold(const T *__restrict__ terms, long stride, int len,
                                                 double *__restrict__ gbeta, long nlinks) {
    const long l = (long)blockIdx.x * BLK + threadIdx.x;
    if (l >= nlinks) return;
    double g = gbeta[l];
    constexpr int U = 8;   // terms loaded ahead of the ordered sum
    int j = len - 1;
    for (; j >= U - 1; j -= U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = terms[(long)(j - u) * stride + l];
#pragma unroll
        for (int u = 0; u < U; u++) g += (double)v[u];
    }
    for (; j >= 0; j--) g += (double)terms[(long)j * stride + l];
    gbeta[l] = g;
}

// dL/dk_r per solid interface node from dL/dbeta of its links (direction
// order): beta = (1 - k)/(1 + k), k = coef * k_r, dbeta/dk_r = -2 coef/(1+k)^2
template <class L>
__global__ __launch_bounds__(BLK) void k_adj_grad(const int32_t *__restrict__ sif,
                                                  const int32_t *__restrict__ soff,
                                                  const int32_t *__restrict__ slinks,
                                                  const int32_t *__restrict__ lnode,
                                                  const uint8_t *__restrict__ ldir,
                                                  const uint32_t *__restrict__ rmask,
                                                  const double *__restrict__ kr,
                                                  const double *__restrict__ nrm,
                                                  const DomDev *__restrict__ doms,
                                                  const double *__restrict__ gbeta, long nsif,
                                                  double *__restrict__ grad) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    if (j >= nsif) return;
    const DomDev D = doms[0];
    const long s = sif[j];
    double gsum = 0.0;
    for (int m = soff[j]; m < soff[j + 1]; m++) {
        const int l = slinks[m];
        const int i = ldir[l];
        const double en = L::ex[i] * nrm[3 * s] + L::ey[i] * nrm[3 * s + 1] + L::ez[i] * nrm[3 * s + 2];
        double coef;
        if (D.scheme == LBM_SV) coef = en > 0 ? en / D.cs2s : 0.0;
        else if (D.scheme == LBM_SPJ) coef = en > 0 ? D.gamma / (D.cs2s * en) : 0.0;
        else if (D.scheme == LBM_ABB) coef = 0.0;
        else coef = en > 0 ? D.gamma * en / D.cs2s : 0.0;
        if (D.mech == LBM_PRECOLL && (rmask[lnode[l]] & (1u << L::opp[i]))) coef /= D.gamma;
        const double kap = coef * kr[s];
        gsum += gbeta[l] * (-2.0 * coef / ((1.0 + kap) * (1.0 + kap)));
    }
    grad[s] = gsum;
}

__global__ void k_zero_i32_adj(int32_t *p) { *p = 0; }

__global__ __launch_bounds__(BLK) void k_adj_zero(double *p, long n) {
    const long i = (long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// The fluid is a fixed point of the step (and its velocity stays exactly 0)
// when every fluid node holds the equilibrium at rest of one common density:
// f_i = w_i rho with rho that of the first fluid node.  Momentum alone is not
// enough: a density difference, or a non-equilibrium part, drives a flow in
// later steps that the adjoint (which recomputes with u = 0) would not see.
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_rest_check(long nf, long S, const T *__restrict__ f,
                                                    const int32_t *__restrict__ nodeof, double rho0,
                                                    int32_t *flag) {
    const long k = (long)blockIdx.x * BLK + threadIdx.x;
    if (k >= nf || nodeof[k] < 0) return;
    double rref = 0.0;
    for (int i = 0; i < L::Q; i++) rref += (double)f[pidx(i, 0, L::Q)] + L::w[i] * rho0;
    bool off = false;
    for (int i = 0; i < L::Q; i++) {
        const double v = (double)f[pidx(i, k, L::Q)] + L::w[i] * rho0;
        off |= !(fabs(v - L::w[i] * rref) <= 1e-9 * fabs(rref));
    }
    if (off) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
template <typename T>
static AdjArgs<T> adj_args(Ctx &c) {
    AdjArgs<T> a;
    a.pin = nullptr;
    a.pout = nullptr;
    a.gin = nullptr;
    a.gout = nullptr;
    a.tasks = c.tasks;
    a.rows = c.rows;
    a.doms = c.doms;
    a.nodeof = c.nodeof;
    a.lbase = c.lbase;
    a.lbeta = (const T *)c.lbeta;
    a.lsrc = nullptr;
    a.gbeta = c.adj.gbeta;
    a.dldc = nullptr;
    a.ntasks = c.n_tasks;
    a.S = c.S;
    return a;
}

template <class L, typename T>
static hipError_t rest_check_impl(Ctx &c, bool *at_rest) {
    hipLaunchKernelGGL(k_zero_i32_adj, dim3(1), dim3(1), 0, c.stream, c.iacc + 5);
    const long nf = c.n_slots;
    if (nf > 0)
        hipLaunchKernelGGL((k_rest_check<L, T>), dim3((nf + BLK - 1) / BLK), dim3(BLK), 0, c.stream,
                           nf, c.S, (const T *)c.f[c.cur], c.nodeof, c.fp64 ? 0.0 : c.p.rho0, c.iacc + 5);
    int32_t flag = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, c.iacc + 5, 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    *at_rest = flag == 0;
    return e;
}

// the kernel durations of one launch bracketed by events ev[0], ev[1] (timed
// adjoint only): waits for it and adds the milliseconds to *acc
static hipError_t add_elapsed(Ctx &c, double *acc) {
    hipError_t e = hipEventSynchronize(c.ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, c.ev[0], c.ev[1]);
    if (e == hipSuccess) *acc += t;
    return e;
}

template <class L, typename T, bool RED, bool TRT>
static hipError_t adjoint_impl(Ctx &c, const double *dldc, double *grad, double *ms) {
    const AdjState &r = c.adj;
    const long nb = (c.n_tasks + BLK / 64 - 1) / (BLK / 64);
    const size_t slot = (size_t)c.QS * c.S;
    AdjArgs<T> a = adj_args<T>(c);
    T *P[2] = {(T *)r.p[0], (T *)r.p[1]};
    const T *ck = (const T *)r.ckpt;
    T *rs[2] = {(T *)r.rst[0], (T *)r.rst[1]};
    // dL/dbeta := 0, lambda(T) from dL/dC_T
    hipLaunchKernelGGL(k_adj_zero, dim3((c.n_links + BLK - 1) / BLK + 1), dim3(BLK), 0, c.stream,
                       r.gbeta, (long)c.n_links);
    a.dldc = dldc;
    a.pout = P[0];
    if (nb > 0) hipLaunchKernelGGL((k_adj_init<L, T, RED>), dim3(nb), dim3(BLK), 0, c.stream, a);
    int cur = 0;
    const int nseg = (int)((r.nsteps + r.ckpt_every - 1) / r.ckpt_every);
    auto seg_len = [&](int sgi) {
        const long t0 = (long)sgi * r.ckpt_every;
        return (int)((r.nsteps - t0) < r.ckpt_every ? (r.nsteps - t0) : r.ckpt_every);
    };
    // recomputation of segment sgi on stream st: state 0 of the segment is
    // its checkpoint, state j > 0 lives in rs[(j - 1) & 1]; stepping from
    // state j records the links' source values of step j into src (the last
    // state's successor is not needed)
    auto recompute = [&](int sgi, hipStream_t st, T *src) -> hipError_t {
        AdjArgs<T> b = a;
        const int len = seg_len(sgi);
        for (int j = 0; j < len; j++) {
            b.gin = j == 0 ? (T *)(ck + (size_t)sgi * slot) : rs[(j - 1) & 1];
            b.gout = j + 1 < len ? rs[j & 1] : nullptr;
            b.lsrc = src + (size_t)j * r.src_stride;
            if (ms) (void)hipEventRecord(c.ev[0], st);
            if (nb > 0) hipLaunchKernelGGL((k_sol_step<L, T, RED, TRT>), dim3(nb), dim3(BLK), 0, st, b);
            if (ms) {
                (void)hipEventRecord(c.ev[1], st);
                hipError_t e = add_elapsed(c, &ms[0]);
                if (e != hipSuccess) return e;
            }
        }
        return hipGetLastError();
    };
    // the transposed steps of segment sgi, last step first, on the context stream
    auto transpose = [&](int sgi, const T *src) -> hipError_t {
        a.gin = nullptr;
        a.gout = nullptr;
        for (int j = seg_len(sgi) - 1; j >= 0; j--) {
            a.lsrc = (T *)src + (size_t)j * r.src_stride;
            a.pin = P[cur];
            a.pout = P[1 - cur];
            if (ms) (void)hipEventRecord(c.ev[0], c.stream);
            if (nb > 0) hipLaunchKernelGGL((k_adj_step<L, T, RED, TRT>), dim3(nb), dim3(BLK), 0, c.stream, a);
            if (ms) {
                (void)hipEventRecord(c.ev[1], c.stream);
                hipError_t e = add_elapsed(c, &ms[1]);
                if (e != hipSuccess) return e;
            }
            cur = 1 - cur;
        }
        if (c.n_links > 0) {
            if (ms) (void)hipEventRecord(c.ev[0], c.stream);
            hipLaunchKernelGGL((k_adj_fold<T>), dim3((c.n_links + BLK - 1) / BLK), dim3(BLK), 0, c.stream, src,
                               (long)r.src_stride, seg_len(sgi), r.gbeta, (long)c.n_links);
            if (ms) {
                (void)hipEventRecord(c.ev[1], c.stream);
                hipError_t e = add_elapsed(c, &ms[2]);
                if (e != hipSuccess) return e;
            }
        }
        return hipGetLastError();
    };
    // With a second source buffer the recomputation of segment sgi - 1 runs
    // on the side stream while the transposed steps of segment sgi run on
    // the context stream: they share no array (the transposed steps read no
    // state), and both kernels are bound by latency rather than bandwidth at
    // the sizes the adjoint is run at.  The timed variant, and a stream under
    // capture, keep everything on the context stream.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c.stream, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
    const bool ovl = !ms && r.lsrc2 && c.have_side && nseg > 1 && cap == hipStreamCaptureStatusNone;
    T *buf[2] = {(T *)r.lsrc, ovl ? (T *)r.lsrc2 : (T *)r.lsrc};
    hipError_t e = hipSuccess;
    if (ovl) e = recompute(nseg - 1, c.stream, buf[(nseg - 1) & 1]);
    for (int sgi = nseg - 1; sgi >= 0 && e == hipSuccess; sgi--) {
        T *src = buf[sgi & 1];
        if (!ovl) {
            e = recompute(sgi, c.stream, src);
            if (e == hipSuccess) e = transpose(sgi, src);
            continue;
        }
        if (sgi > 0) {
            // after all work so far on the context stream: the recomputation
            // of segment sgi (whose states it reuses) and the transposed steps
            // of segment sgi + 1 (which read the buffer it fills)
            if ((e = hipEventRecord(c.ev_adj[0], c.stream)) != hipSuccess) break;
            if ((e = hipStreamWaitEvent(c.side, c.ev_adj[0], 0)) != hipSuccess) break;
            if ((e = recompute(sgi - 1, c.side, buf[(sgi - 1) & 1])) != hipSuccess) break;
            if ((e = hipEventRecord(c.ev_adj[1], c.side)) != hipSuccess) break;
        }
        if ((e = transpose(sgi, src)) != hipSuccess) break;
        // the next segment's transposed steps wait for its recomputation
        if (sgi > 0) e = hipStreamWaitEvent(c.stream, c.ev_adj[1], 0);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_zero, dim3((c.N + BLK - 1) / BLK), dim3(BLK), 0, c.stream, grad, c.N);
    if (c.n_sif > 0)
        hipLaunchKernelGGL((k_adj_grad<L>), dim3((c.n_sif + BLK - 1) / BLK), dim3(BLK), 0, c.stream,
                           c.sif, c.soff, c.slinks, c.lnode, c.ldir, c.rmask, c.kr, c.nrm, c.doms,
                           (const double *)r.gbeta, (long)c.n_sif, grad);
    return hipGetLastError();
}

hipError_t launch_rest_check(Ctx &c, bool *at_rest) {
    if (c.Q == 9) return c.fp64 ? rest_check_impl<D2Q9, double>(c, at_rest) : rest_check_impl<D2Q9, float>(c, at_rest);
    return c.fp64 ? rest_check_impl<D3Q19, double>(c, at_rest) : rest_check_impl<D3Q19, float>(c, at_rest);
}

template <class L, typename T>
static hipError_t adjoint_set(Ctx &c, const double *dldc, double *grad, double *ms) {
    // the collision and the solute set are compile-time variants: a runtime
    // TRT branch costs the BGK transpose a wave of occupancy
    const bool trt = c.p.collision == LBM_TRT;
    if (trt) return c.red ? adjoint_impl<L, T, true, true>(c, dldc, grad, ms) : adjoint_impl<L, T, false, true>(c, dldc, grad, ms);
    return c.red ? adjoint_impl<L, T, true, false>(c, dldc, grad, ms) : adjoint_impl<L, T, false, false>(c, dldc, grad, ms);
}

hipError_t launch_adjoint(Ctx &c, const double *dldc, double *grad, double *ms) {
    if (c.Q == 9) return c.fp64 ? adjoint_set<D2Q9, double>(c, dldc, grad, ms) : adjoint_set<D2Q9, float>(c, dldc, grad, ms);
    return c.fp64 ? adjoint_set<D3Q19, double>(c, dldc, grad, ms) : adjoint_set<D3Q19, float>(c, dldc, grad, ms);
}

}  // namespace lbm
