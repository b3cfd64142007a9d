// lbm_step.hip -- the per-step kernels of the reactive lattice Boltzmann method.
//
// One time step is two launches on the context stream:
//   k_step       one wavefront per task (up to 64 consecutive fluid nodes of
//                one x-row).  Fluid: pull-stream with halfway bounce-back,
//                moments, Guo-forced BGK or TRT.  Solute: pull-stream, inlet/outlet
//                planes, the general reactive boundary condition on every link
//                that enters from a solid node, advection-diffusion BGK with
//                the rest-fraction weights (on the fluid's velocity set, or on
//                D2Q5 / D3Q7 when RED: the solute loops then visit the set's
//                directions only, at compile time); writes the exchange q of each
//                reactive link and credits precipitation (q < 0) to the fluid
//                node's phi.  The task's links are one range (by direction,
//                then lane): their betas are fetched into LDS in one pass
//                ahead of the loads, each link's q replaces its beta there,
//                and the range is stored in one pass.
//                Compile-time variants: TRT collision, the reduced solute set
//                (RED), the open channel's inflow/outflow faces (OPEN) and a
//                per-node C_eq read per link (CEQ); the rarely used ones only
//                at four waves per workgroup, so that the common kernel keeps
//                its registers.
//
// The neighbour classification is written out here rather than taken from
// classify() (lbm_task.hpp, used by the adjoint kernels): the compiler
// schedules the inlined helper differently and the step ran 1.5x slower.
//   k_phi_solid  per solid interface node: dissolution (q > 0) charged to its
//                phi in link order, and the step's total wall exchange.
//
// All loads of a node (both lattices) are issued before any arithmetic, so a
// wavefront keeps 2Q loads in flight; each population value is read once by
// k_step.  Arithmetic is FP64 in both storage precisions: near a steady state
// every node rounds the same moment sums and equilibria the same way at every
// step, and in FP32 that rounding acts as a fixed spurious body force and
// source (velocity errors of a few 1e-5 after ~10^4 steps in a channel).
#include "lbm_internal.hpp"
#include "lbm_task.hpp"

namespace lbm {

// WV wavefronts (tasks) per workgroup; remap != 0 keeps runs of consecutive
// tiles on one XCD.  FP32 storage asks for 4 waves per SIMD (at most 128
// VGPRs): the extra wave hides more memory latency than a spill would cost
// (256^3 sphere packing: 732 -> 660 us when it was first tried).
template <class L, typename T, int WV, bool TRT, bool RED, bool OPEN, bool CEQ>
__global__ __launch_bounds__(64 * WV, sizeof(T) == 4 ? 4 : 1) void k_step(StepArgs<T> a, long nblocks,
                                                                         int remap) {
    using R = double;
    constexpr int Q = L::Q;
    // the solute set, and the storage slot of each of its directions
    constexpr uint32_t SM = sol_mask<L, RED>();
    constexpr int QS = __builtin_popcount(SM);
    const long tile = remap ? xcd_tile(blockIdx.x, nblocks) : (long)blockIdx.x;
    const int t = __builtin_amdgcn_readfirstlane((int)(tile * WV) + (int)(threadIdx.x >> 6));
    if (t >= a.ntasks) return;
    // phase change: nothing to do once an earlier step of this batch crossed
    // a threshold (the host runs the event pass and repeats from there)
    if (a.evflag) {
        const unsigned long long w = *a.evflag;
        if ((int)(w >> 32) == a.evbatch && (int)(unsigned)w < a.evidx) return;
    }
    const int lane = threadIdx.x & 63;
    const Task tk = a.tasks[t];
    // by value, read before the first store: loads of a uniform address that no
    // store can precede stay on the scalar unit.  A single-domain context's
    // record does not wait for the task.
    DomDev D = a.doms[0];
    if (a.ndom > 1) D = a.doms[tk.dom];
    const Box b = D.box;
    const long S = a.S;
    const int W = D.W;
    const RowWord *__restrict__ rows = a.rows + D.word_off;
    const int y0 = tk.y0, z = tk.z;
    const int cnt = tk.cnt & 255, nr = tk.cnt >> 8;
    const int ax = b.inlet_axis;

    // ---- the row words of every row this task pulls from: a table of the
    // rows y0 - 1 .. y0 + nr of the planes z - 1 .. z + 1 (one plane in 2D);
    // lane j holds word (j % W) of table row (j / W); other lanes read them
    // with cross-lane shuffles ----
    const int TY = nr + 2;
    const int NSL = (L::DIM == 3 ? 3 : 1) * TY;
    const int wlo = tk.wlo, nwd = tk.nwd;   // window of words of each table row
    const bool slots_fit = NSL * nwd <= 64;
    unsigned long long wm = 0ull;
    int wpb = 0;
    if (slots_fit && lane < NSL * nwd) {
        // small quotients by float reciprocal (exact: the dividend is offset by
        // one half, far from a multiple of the divisor)
        const int sl = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)nwd));
        const int w = wlo + (lane - sl * nwd);
        const int sq = (int)(((float)sl + 0.5f) * __builtin_amdgcn_rcpf((float)TY));
        int yy = y0 - 1 + (sl - sq * TY), zz = L::DIM == 3 ? z - 1 + sq : z, xx = 0, fc;
        if (wrap_site(b, xx, yy, zz, &fc)) {
            const RowWord rw = rows[(long)(yy + b.ny * zz) * W + w];
            wm = rw.mask;
            wpb = rw.pb;
        }
    }
    // every lane stays active through the shuffles below; lanes past the end
    // of the task classify the task's first node and leave before any load
    const bool active = lane < cnt;
    const int k = tk.k0 + (active ? lane : 0);
    // the lane's row: the last of the task's rows that starts at or before k
    // (a row's first compact index is the base of its first word)
    int ry = 0;
    for (int j = 1; j < nr; j++) {
        const int pbj = __shfl(wpb, ((L::DIM == 3 ? TY : 0) + j + 1) * nwd, 64);
        if (k >= pbj) ry = j;
    }
    const int y = y0 + ry;
    const int n = a.nodeof[k];
    const int lb = a.lbase[k];  // the links of the nodes before k (lane 0: the task's first link)
    const int x = (int)(n - D.node_off) - (tk.row + ry) * b.nx;

    // ---- neighbour classification (shared by both lattices) ----
    // A pull along i reads site (x, y, z) - e_i, which lies past a face of the
    // box only if the node is on that face: the faces the node lies on give,
    // once per node, the directions that leave the box (bit masks).
    constexpr uint32_t PX = dir_mask<L>(0, 1), NX = dir_mask<L>(0, -1);
    constexpr uint32_t PY = dir_mask<L>(1, 1), NY = dir_mask<L>(1, -1);
    constexpr uint32_t PZ = dir_mask<L>(2, 1), NZ = dir_mask<L>(2, -1);
    const uint32_t fx = (x == 0 ? PX : 0u) | (x == b.nx - 1 ? NX : 0u);
    const uint32_t fy = (y == 0 ? PY : 0u) | (y == b.ny - 1 ? NY : 0u);
    const uint32_t fz = (z == 0 ? PZ : 0u) | (z == b.nz - 1 ? NZ : 0u);
    // out of a non-periodic box; an x wrap that shifts the row (tilted torus)
    const uint32_t outm = (b.per[0] ? 0u : fx) | (b.per[1] ? 0u : fy) | (b.per[2] ? 0u : fz);
    const uint32_t shiftm = (b.per[0] && b.shift != 0) ? fx : 0u;
    // across the inlet (cross) or outlet (cross and cross_hi) plane
    uint32_t cross = 0u, cross_hi = 0u;
    if (ax >= 0) {
        const uint32_t f = ax == 0 ? fx : (ax == 1 ? fy : fz);
        const uint32_t pm = ax == 0 ? PX : (ax == 1 ? PY : PZ);
        cross = f;
        cross_hi = f & ~pm;
    }
    // the three x offsets of a pull (x + 1, x, x - 1 for e_x = -1, 0, 1):
    // column of the table (-1: outside it) and bit within the row word.  x
    // wraps within the row when periodic; a wrap that shifts the row, or a
    // word outside the table, goes through the row words in memory.
    int tcol[3];
    unsigned long long tbit[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        const int xn = x + 1 - v;
        const int xw = !b.per[0] ? xn : (xn < 0 ? xn + b.nx : (xn >= b.nx ? xn - b.nx : xn));
        const int xs = min(max(xw, 0), b.nx - 1);
        const int tw = (xs >> 6) - wlo;
        tcol[v] = (slots_fit && tw >= 0 && tw < nwd) ? ry * nwd + tw : -1;
        tbit[v] = 1ull << (xs & 63);
    }
    int kk[Q];
    uint32_t solidnb = 0u;
    kk[0] = k;
    // The common case, decided once per wavefront: every pull of every lane
    // is resolved by the table (no box face, no shifted wrap, all three x
    // columns inside it).  Then the classification is straight-line selects;
    // otherwise each direction takes the general path.
    const bool tab_ok = slots_fit && outm == 0u && shiftm == 0u && tcol[0] >= 0 && tcol[1] >= 0 &&
                        tcol[2] >= 0;
    if (__ballot(!tab_ok) == 0ull) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int v = L::ex[i] + 1;
            const int src = ((L::DIM == 3 ? (1 - L::ez[i]) * TY : 0) + 1 - L::ey[i]) * nwd + tcol[v];
            const unsigned lo = __shfl((unsigned)(wm & 0xffffffffull), src, 64);
            const unsigned hi = __shfl((unsigned)(wm >> 32), src, 64);
            const int pb = __shfl(wpb, src, 64);
            const unsigned long long m = ((unsigned long long)hi << 32) | lo;
            const unsigned long long bit = tbit[v];
            kk[i] = (m & bit) ? pb + __popcll(m & (bit - 1ull)) : -1;
            if (kk[i] == -1) solidnb |= 1u << i;
        }
    } else {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int v = L::ex[i] + 1;
            const bool in_tab = tcol[v] >= 0;
            // the shuffles run on every lane: a shuffle reads zero from a lane
            // that is inactive at that point
            const int src = in_tab ? ((L::DIM == 3 ? (1 - L::ez[i]) * TY : 0) + 1 - L::ey[i]) * nwd + tcol[v] : 0;
            const unsigned lo = __shfl((unsigned)(wm & 0xffffffffull), src, 64);
            const unsigned hi = __shfl((unsigned)(wm >> 32), src, 64);
            const int pb = __shfl(wpb, src, 64);
            if (outm & (1u << i)) {
                kk[i] = -2;
            } else if (!in_tab || (shiftm & (1u << i))) {
                kk[i] = nb_compact(rows, W, b, x - L::ex[i], y - L::ey[i], z - L::ez[i]);
            } else {
                const unsigned long long m = ((unsigned long long)hi << 32) | lo;
                const unsigned long long bit = tbit[v];
                kk[i] = (m & bit) ? pb + __popcll(m & (bit - 1ull)) : -1;
            }
            if (kk[i] == -1) solidnb |= 1u << i;
        }
    }
    const uint32_t rbc = active ? (solidnb & ~cross & SM) : 0u;

    // ---- the task's reactive links: one range from lbase of its first node,
    // ordered by direction, then by lane (a link's index is the task's base,
    // the links of the earlier directions, and the lanes below holding the
    // same direction).  Their coefficients beta = (1 - k_i)/(1 + k_i) are
    // fetched straight into LDS in link order (no VGPR waits on them); each
    // link's exchange later replaces its coefficient there, and the whole
    // range is stored at once at the end ----
    constexpr int NW = (int)(sizeof(T) / 4);
    __shared__ uint32_t slink[WV][NW][64 * (QS - 1)];
    const int wv = threadIdx.x >> 6;
    const int lt = __builtin_amdgcn_readfirstlane(lb);
    const unsigned long long below = (1ull << lane) - 1ull;
    int nlt = 0;
#pragma unroll
    for (int i = 1; i < Q; i++)
        if ((SM >> i) & 1u) nlt += __popcll(__ballot((rbc >> i) & 1u));
    for (int c = 0; c < nlt; c += 64) {
        if (c + lane < nlt) {
            const uint32_t *p = (const uint32_t *)(a.lbeta + lt + c + lane);
#pragma unroll
            for (int w = 0; w < NW; w++)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(p + w),
                                                 (__attribute__((address_space(3))) void *)&slink[wv][w][c],
                                                 4, 0, 0);
        }
    }
    if (!active) return;
    // the solid fraction of an interface node, read now so that its latency
    // hides behind the population loads (updated at the end)
    const double phi_in = rbc ? a.phif[k] : 0.0;

    // ---- loads: Q fluid + QS solute values per node ----
    const long obf = blk0(k, Q), obg = blk0(k, QS);   // the node's own slot 0
    T fv[Q], gv[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        // fluid neighbour: pull along i; solid or box face: own value along opp(i)
        fv[i] = a.fin[kk[i] >= 0 ? pidx(i, kk[i], Q) : obf + 64 * L::opp[i]];
    }
#pragma unroll
    for (int i = 0; i < Q; i++) {
        if (!((SM >> i) & 1u)) continue;
        int e = kk[i];
        if (cross & (1u << i)) {
            if (cross_hi & (1u << i)) {
                // zero-gradient outlet: the same direction one site back
                // along the inlet axis, inside the outlet plane
                e = nb_compact(rows, W, b, x - L::ex[i] - (ax == 0),
                               y - L::ey[i] - (ax == 1), z - L::ez[i] - (ax == 2));
            } else {
                e = -1;  // inlet: the node's own value along opp(i) (the
                         // population leaving there); the incoming one is set below
            }
        }
        // fluid neighbour: pull; solid or box face: own value along opp(i)
        gv[i] = a.gin[e >= 0 ? pidx(sol_slot(SM, i), e, QS) : obg + 64 * sol_slot(SM, L::opp[i])];
    }

    // ---- fluid: moments and Guo-forced BGK ----
    R fp[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) fp[i] = (R)fv[i];
    // open channel: the box faces of the inlet axis carry the plug inflow
    // (bounce-back from a wall moving with u_in) and the outlet density
    // (anti-bounce-back at rho_out); values are deviations from w rho0.  A
    // separate instantiation: in the others it would cost registers (spills)
    if (OPEN && D.fopen && cross) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (!(cross & (1u << i))) continue;
            const R ea = R(ax == 0 ? L::ex[i] : (ax == 1 ? L::ey[i] : L::ez[i]));
            if (cross_hi & (1u << i)) fp[i] = -fp[i] + R(2) * R(L::w[i]) * (D.rho_out - D.rho0);
            else fp[i] = fp[i] + R(6) * R(L::w[i]) * D.rho_out * (ea * D.u_in);
        }
    }
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        drho += fp[i];
        if (L::ex[i]) jx += L::ex[i] > 0 ? fp[i] : -fp[i];
        if (L::ey[i]) jy += L::ey[i] > 0 ? fp[i] : -fp[i];
        if (L::ez[i]) jz += L::ez[i] > 0 ? fp[i] : -fp[i];
    }
    const R rho = D.rho0 + drho;
    const R irho = R(1) / rho;
    // rho u = j + F/2 enters the first-order equilibrium term directly, so the
    // equilibrium carries exactly the momentum of the node
    const R mx = jx + R(0.5) * D.F[0], my = jy + R(0.5) * D.F[1], mz = jz + R(0.5) * D.F[2];
    const R ux = mx * irho, uy = my * irho, uz = mz * irho;
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * D.F[0] + uy * D.F[1] + uz * D.F[2];
    // f* = f + om (f_eq - f) + ff S, a direction and its opposite together:
    // e.u, e.m and e.F change sign with e, so f*_(i, opp i) = (1 - om) f + A
    // +- B with the even part A = w (om (drho + rho (9/2 (e.u)^2 - 3/2 u.u))
    // + ff (9 (e.u)(e.F) - 3 u.F)) and the odd part B = 3 w (om e.m + ff e.F).
    // A is evaluated as w (base + e.u (9/2 om rho e.u + 9 ff e.F)) with the
    // node's base = om (drho - 3/2 rho u.u) - 3 ff u.F: two fused
    // multiply-adds per pair on top of e.u
    const R om = D.omega_f, ff = D.force_fac, om1 = R(1) - om;
    const R base = om * (drho - R(1.5) * rho * uu) - R(3) * ff * uF;
    const R c45 = R(4.5) * om * rho;
    __builtin_nontemporal_store((T)(om1 * fp[0] + R(L::w[0]) * base), &a.fout[obf]);
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (L::opp[i] < i) continue;
        const int o = L::opp[i];
        const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
        const R em = R(L::ex[i]) * mx + R(L::ey[i]) * my + R(L::ez[i]) * mz;
        const R eF = R(L::ex[i]) * D.F[0] + R(L::ey[i]) * D.F[1] + R(L::ez[i]) * D.F[2];
        const R wi = R(L::w[i]);
        const R A = wi * (base + eu * (c45 * eu + R(9) * ff * eF));
        if constexpr (TRT) {
            // TRT: the odd parts (f_i - f_o)/2, e.m and e.F relax with the
            // second rate, the even ones with om
            const R B = R(3) * wi * (D.omega_fm * em + D.force_fac_m * eF);
            const R hp = R(0.5) * om * (fp[i] + fp[o]), hm = R(0.5) * D.omega_fm * (fp[i] - fp[o]);
            __builtin_nontemporal_store((T)(fp[i] - hp - hm + (A + B)), &a.fout[obf + 64 * i]);
            __builtin_nontemporal_store((T)(fp[o] - hp + hm + (A - B)), &a.fout[obf + 64 * o]);
        } else {
            const R B = R(3) * wi * (om * em + ff * eF);
            __builtin_nontemporal_store((T)(om1 * fp[i] + (A + B)), &a.fout[obf + 64 * i]);
            __builtin_nontemporal_store((T)(om1 * fp[o] + (A - B)), &a.fout[obf + 64 * o]);
        }
    }

    // The task's coefficients were fetched into LDS by global-to-LDS loads,
    // which the compiler does not order before LDS reads.  They were issued
    // before the fluid loads, and the fluid stores above consumed every fluid
    // load: vector memory operations complete in order, so those loads' waits
    // cover the coefficients.  This barrier keeps the compiler from moving an
    // LDS read of them above the fluid stores (an explicit wait for all vector
    // memory operations here would also wait for the stores: 8 us slower).
    asm volatile("" ::: "memory");
    // ---- solute: plane faces, reactive links, collision ----
    // Inlet: the equilibrium at C_in for the populations entering across the
    // plane.  The mass a plane link brings in is the incoming value minus the
    // node's own value leaving along the opposite direction (at the inlet
    // that one was loaded into gv; at the outlet gv holds the zero-gradient
    // copy, and the own value is read here: outlet nodes only).  Each wavefront
    // with plane nodes adds its sums (fixed shuffle order) to its task's slots.
    if (ax >= 0) {
        R xin = R(0), xout = R(0);
        if (cross) {
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if (!((SM >> i) & 1u) || !(cross & (1u << i))) continue;
                if (cross_hi & (1u << i)) {
                    xout += (R)gv[i] - (R)a.gin[obg + 64 * sol_slot(SM, L::opp[i])];
                } else {
                    const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
                    const R gin = sol_w<L>(D, i) * (D.c_in - D.c_ref) + sol_w<L>(D, i) * D.c_in * eu * D.inv_cs2s;
                    xin += gin - (R)gv[i];
                    gv[i] = (T)gin;
                }
            }
        }
        if (__ballot(cross != 0u)) {
            xin = wave_sum(xin);
            xout = wave_sum(xout);
            if (lane == 0) {
                a.xio[t] += xin;
                a.xio[a.task_cap + t] += xout;
            }
        }
    }
    // general reactive boundary condition on each link entering from a solid
    // node (direction order):
    //   g_in = k/(1+k) 2 w_i C_eq + (1-k)/(1+k) g_src = (1 - beta) w_i C_eq + beta g_src
    // (deviation form: C_eq - C_ref, since beta - 1 = -2 k/(1+k)).  g_src is the
    // population moving toward the wall: the one pulled into this node along the
    // opposite direction (pre-collision mechanics), or the node's own
    // post-collision value (link-wise mechanics, and the one-node-gap fallback,
    // whose beta already carries k/gamma).  q = g_in - g_out crossed the link.
    if (rbc) {
        double sneg = 0.0;
        int off = 0;
        // w_i C_eq = L::w[i] (wsc C_eq) with a uniform C_eq: one value held in
        // registers of the wavefront (the loop's blocks otherwise reload the
        // two factors from spilled scalar registers in every direction)
        const R wceq = D.wsc * D.ceq_dev;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (!((SM >> i) & 1u)) continue;
            const unsigned long long bal = __ballot((rbc >> i) & 1u);
            const int pos = off + __popcll(bal & below);   // position in the task's range
            off += __popcll(bal);
            if (rbc & (1u << i)) {
                const int o = L::opp[i];
                const R own = (R)gv[i];  // a link direction loaded the node's own value along o
                const R srcv = (D.mech == LBM_PRECOLL && !(rbc & (1u << o))) ? (R)gv[o] : own;
                T bt;
                if constexpr (NW == 1) {
                    bt = __builtin_bit_cast(T, slink[wv][0][pos]);
                } else {
                    const unsigned long long lo = slink[wv][0][pos], hi = slink[wv][NW - 1][pos];
                    bt = __builtin_bit_cast(T, lo | (hi << 32));
                }
                const R beta = (R)bt;
                // w_i C_eq with the link's C_eq: per solid node (a separate
                // instantiation), or uniform
                R wc = R(L::w[i]) * wceq;
                if constexpr (CEQ) wc = sol_w<L>(D, i) * (R)a.lceq[lt + pos];
                // (1 - beta) w C_eq + beta g_src: exactly g_src at beta = 1
                const R g = (R(1) - beta) * wc + beta * srcv;
                const T qv = (T)(g - own);
                if constexpr (NW == 1) {
                    slink[wv][0][pos] = __builtin_bit_cast(uint32_t, qv);
                } else {
                    const unsigned long long qb = __builtin_bit_cast(unsigned long long, qv);
                    slink[wv][0][pos] = (uint32_t)qb;
                    slink[wv][NW - 1][pos] = (uint32_t)(qb >> 32);
                }
                sneg -= (double)(qv < T(0) ? qv : T(0));
                gv[i] = (T)g;
            }
        }
        if (sneg != 0.0) a.phif[k] = phi_in + D.vma * sneg;
        // phase change: a node at or past the precipitation threshold marks
        // the step (every interface node's value is checked, changed or not)
        if (a.evflag && (sneg != 0.0 ? phi_in + D.vma * sneg : phi_in) >= 1.0)
            *a.evflag = ((unsigned long long)(unsigned)a.evbatch << 32) | (unsigned)a.evidx;
    }
    // the task's exchanges, stored in link order by the active lanes
    for (int j = lane; j < nlt; j += cnt) {
        if constexpr (NW == 1) {
            a.lq[lt + j] = __builtin_bit_cast(T, slink[wv][0][j]);
        } else {
            const unsigned long long lo = slink[wv][0][j], hi = slink[wv][NW - 1][j];
            a.lq[lt + j] = __builtin_bit_cast(T, lo | (hi << 32));
        }
    }
    R dC = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++)
        if ((SM >> i) & 1u) dC += (R)gv[i];
    const R C = D.c_ref + dC;
    // g* = g + omg (g_eq - g), g_eq = ws (dC + C e.u / c_s^2): in pairs as
    // above, (1 - omg) g + As +- Bs with As = omg ws dC, Bs = omg ws C e.u / c_s^2
    // TRT: the even parts relax with omega_gs (BGK: omega_gs = omg)
    // the moving weights are w_i wsc: with the node's Cw = omg C wsc / c_s^2
    // and Aw = omg wsc dC (oms for TRT), As = w_i Aw and Bs = w_i Cw e.u
    const R omg = D.omega_g, omg1 = R(1) - omg, oms = D.omega_gs;
    const R Cw = omg * C * D.inv_cs2s * D.wsc;
    const R Aw = (TRT ? oms : omg) * D.wsc * dC;
    __builtin_nontemporal_store((T)((R(1) - oms) * (R)gv[0] + oms * sol_w<L>(D, 0) * dC), &a.gout[obg]);
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (L::opp[i] < i || !((SM >> i) & 1u)) continue;
        const int o = L::opp[i];
        const long si = obg + 64 * sol_slot(SM, i), so = obg + 64 * sol_slot(SM, o);
        const R eu = R(L::ex[i]) * ux + R(L::ey[i]) * uy + R(L::ez[i]) * uz;
        const R wi = R(L::w[i]);
        const R Bs = (wi * Cw) * eu;
        const R As = wi * Aw;
        if constexpr (TRT) {
            const R gi = (R)gv[i], go = (R)gv[o];
            const R hs = R(0.5) * oms * (gi + go), ha = R(0.5) * omg * (gi - go);
            __builtin_nontemporal_store((T)(gi - hs - ha + (As + Bs)), &a.gout[si]);
            __builtin_nontemporal_store((T)(go - hs + ha + (As - Bs)), &a.gout[so]);
        } else {
            __builtin_nontemporal_store((T)(omg1 * (R)gv[i] + (As + Bs)), &a.gout[si]);
            __builtin_nontemporal_store((T)(omg1 * (R)gv[o] + (As - Bs)), &a.gout[so]);
        }
    }
}

// dissolution side of the solid fraction, per solid interface node, links in
// ascending direction order; also the step's total exchange, added to this
// workgroup's own slot xpart[tile] (no atomics: the slots are folded
// into the running total when it is read).  With up to 8 links per node a
// thread takes a node and loads its link ids, then its exchanges.  With the
// 18 of D3Q19 (4.7 on average in a packing) most of those loads would run
// with few lanes active, so a wavefront takes 64 consecutive solid nodes,
// whose links are one contiguous range of the solid-side list: it reads that
// range coalesced and gathers the exchanges of up to PCH * 64 links at a time
// into LDS (every lane loading one link per round), and each lane then sums
// its own node's links from there in order.  Both sum in the same order.
template <class L, typename T, bool RED>
__global__ __launch_bounds__(BLK) void k_phi_solid(const int32_t *__restrict__ soff,
                                                   const int32_t *__restrict__ slinks,
                                                   const int32_t *__restrict__ sdom,
                                                   const DomDev *__restrict__ doms,
                                                   const T *__restrict__ lq, double *__restrict__ phis,
                                                   long nsif, double *__restrict__ xpart, int ndom,
                                                   unsigned long long *evflag, int evbatch, int evidx,
                                                   int remap) {
    constexpr int M = __builtin_popcount(sol_mask<L, RED>()) - 1;
    if (evflag) {   // as in the fused kernel (the value is the same for every thread)
        const unsigned long long w = *evflag;
        if ((int)(w >> 32) == evbatch && (int)(unsigned)w < evidx) return;
    }
    // with remap each XCD takes a contiguous range of solid nodes: the lines
    // of exchanges that neighbouring solid nodes (and those of the next
    // planes) gather stay in that XCD's L2, which cuts the kernel's HBM reads
    // to about its algorithmic bytes
    const long tile = remap ? xcd_tile(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    double tot = 0.0;
    if constexpr (M <= 8) {
        // few links per node (D2Q9, D2Q5, D3Q7): one thread per node loads
        // all its link ids, then all its exchanges, before the ordered sum
        const long j = tile * BLK + threadIdx.x;
        if (j < nsif) {
            const int k0 = soff[j], nk = soff[j + 1] - k0;
            const double ph = phis[j];   // read now: its latency hides behind the gathers
            int li[M];
#pragma unroll
            for (int m = 0; m < M; m++) li[m] = m < nk ? slinks[k0 + m] : -1;
            T qv[M];
#pragma unroll
            for (int m = 0; m < M; m++) qv[m] = li[m] >= 0 ? lq[li[m]] : T(0);
            double pos = 0.0;
#pragma unroll
            for (int m = 0; m < M; m++) {
                const double v = (double)qv[m];
                tot += v;
                if (v > 0.0) pos += v;
            }
            const double pn = ph - doms[ndom > 1 ? sdom[j] : 0].vma * pos;
            phis[j] = pn;
            // phase change: at or past the dissolution threshold
            if (evflag && pn <= 0.0) *evflag = ((unsigned long long)(unsigned)evbatch << 32) | (unsigned)evidx;
        }
    } else {
        constexpr int PCH = 8;
        __shared__ T sq[BLK / 64][64 * PCH];
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const long j0 = tile * BLK + wv * 64, j = j0 + lane;
        if (j0 < nsif) {
            const bool act = j < nsif;
            // lanes past the end read the last node's entries (no branches around
            // the loads: the solid fraction's latency then hides behind the gathers)
            const long jc = act ? j : nsif - 1;
            const int kb0 = soff[jc], ke0 = soff[jc + 1];
            const double ph = phis[jc];
            const int kb = act ? kb0 : 0, ke = act ? ke0 : 0;
            const int last = (int)(nsif - j0 < 64 ? nsif - j0 : 64) - 1;
            const int s0 = __builtin_amdgcn_readfirstlane(kb);
            const int ns = __builtin_amdgcn_readlane(ke, last) - s0;   // links of the wavefront's nodes
            const int mb = kb - s0, me = ke - s0;                       // this lane's node, in that range
            double pos = 0.0;
            for (int c0 = 0; c0 < ns; c0 += 64 * PCH) {
                int li[PCH];
#pragma unroll
                for (int r = 0; r < PCH; r++) {
                    const int p = c0 + r * 64 + lane;
                    li[r] = p < ns ? slinks[s0 + p] : -1;
                }
                T qv[PCH];
#pragma unroll
                for (int r = 0; r < PCH; r++) qv[r] = li[r] >= 0 ? lq[li[r]] : T(0);
                // reads of the previous round are done (LDS operations of one
                // wavefront complete in order)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int r = 0; r < PCH; r++) sq[wv][r * 64 + lane] = qv[r];
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const int lo = mb > c0 ? mb : c0, hi = me < c0 + 64 * PCH ? me : c0 + 64 * PCH;
#pragma unroll
                for (int m = 0; m < M; m++) {
                    if (lo + m < hi) {
                        const double v = (double)sq[wv][lo + m - c0];
                        tot += v;
                        if (v > 0.0) pos += v;
                    }
                }
            }
            if (act) {
                const double pn = ph - doms[ndom > 1 ? sdom[j] : 0].vma * pos;
                phis[j] = pn;
                // phase change: at or past the dissolution threshold
                if (evflag && pn <= 0.0) *evflag = ((unsigned long long)(unsigned)evbatch << 32) | (unsigned)evidx;
            }
        }
    }
    tot = block_sum(tot);
    if (threadIdx.x == 0 && tot != 0.0) xpart[tile] += tot;
}

template <typename T>
static StepArgs<T> step_args(Ctx &c) {
    StepArgs<T> a;
    a.fin = (const T *)c.f[c.cur];
    a.fout = (T *)c.f[1 - c.cur];
    a.gin = (const T *)c.g[c.cur];
    a.gout = (T *)c.g[1 - c.cur];
    a.tasks = c.tasks;
    a.rows = c.rows;
    a.doms = c.doms;
    a.nodeof = c.nodeof;
    a.lbase = c.lbase;
    a.lbeta = (const T *)c.lbeta;
    a.lq = (T *)c.lq;
    a.phif = c.phif;
    a.lceq = (const T *)c.lceq;
    a.xio = c.xio;
    a.evflag = c.p.phase_change ? (unsigned long long *)(c.iacc + 16) : nullptr;
    a.evbatch = c.evbatch;
    a.evidx = c.evidx;
    a.task_cap = c.task_cap;
    a.ntasks = c.n_tasks;
    a.ndom = c.ndom;
    a.S = c.S;
    return a;
}

// An open channel or a per-node C_eq runs the 4-wave tile only (its launch
// uses that grid).
template <class L, typename T, bool TRT, bool RED>
static void launch_k_step(int wv, long nb, hipStream_t st, const StepArgs<T> &args, int rm, bool open,
                          bool ceq) {
    if (open || ceq) {
        if (open && ceq)
            hipLaunchKernelGGL((k_step<L, T, 4, TRT, RED, true, true>), dim3(nb), dim3(256), 0, st, args, nb, rm);
        else if (open)
            hipLaunchKernelGGL((k_step<L, T, 4, TRT, RED, true, false>), dim3(nb), dim3(256), 0, st, args, nb, rm);
        else
            hipLaunchKernelGGL((k_step<L, T, 4, TRT, RED, false, true>), dim3(nb), dim3(256), 0, st, args, nb, rm);
        return;
    }
    switch (wv) {
    case 1: hipLaunchKernelGGL((k_step<L, T, 1, TRT, RED, false, false>), dim3(nb), dim3(64), 0, st, args, nb, rm); break;
    case 2: hipLaunchKernelGGL((k_step<L, T, 2, TRT, RED, false, false>), dim3(nb), dim3(128), 0, st, args, nb, rm); break;
    case 8: hipLaunchKernelGGL((k_step<L, T, 8, TRT, RED, false, false>), dim3(nb), dim3(512), 0, st, args, nb, rm); break;
    default: hipLaunchKernelGGL((k_step<L, T, 4, TRT, RED, false, false>), dim3(nb), dim3(256), 0, st, args, nb, rm); break;
    }
}

// One step.  The exchanges alternate between two buffers, so that with
// `overlap` the solid-side kernel of this step runs on the side stream while
// the next step's fused kernel (which writes the other buffer) runs on the
// context stream; a fused kernel waits only for the solid-side kernel that
// read its buffer two steps before.  The solid-side kernel touches the solid
// fractions of solid nodes only, the fused kernel those of fluid nodes.
template <class L, typename T>
static hipError_t step_impl(Ctx &c, hipEvent_t *ev, bool overlap) {
    hipError_t e = hipSuccess;
    const int b = c.lq_next;
    if (c.phi_pending[b]) {
        e = hipStreamWaitEvent(c.stream, c.ev_phi[b], 0);
        if (e != hipSuccess) return e;
        c.phi_pending[b] = false;
    }
    c.lq = c.lqb[b];
    const StepArgs<T> args = step_args<T>(c);
    if (ev) (void)hipEventRecord(ev[0], c.stream);
    if (c.n_tasks > 0) {
        // an open channel or a per-node C_eq (all domains alike) takes the 4-wave tile
        const bool open = c.p.fluid_open != 0, ceq = c.lceq != nullptr;
        const int wv = (open || ceq) ? 4 : c.cfg.wg_waves;
        const long nb = (c.n_tasks + wv - 1) / wv;
        const int rm = c.cfg.xcd_remap;
        // TRT and the reduced solute set are separate instantiations: TRT's
        // extra terms would cost the BGK kernel registers (every domain of a
        // context shares both choices)
        const bool trt = c.p.collision == LBM_TRT;
        if (trt && c.red) launch_k_step<L, T, true, true>(wv, nb, c.stream, args, rm, open, ceq);
        else if (trt) launch_k_step<L, T, true, false>(wv, nb, c.stream, args, rm, open, ceq);
        else if (c.red) launch_k_step<L, T, false, true>(wv, nb, c.stream, args, rm, open, ceq);
        else launch_k_step<L, T, false, false>(wv, nb, c.stream, args, rm, open, ceq);
        e = hipGetLastError();
    }
    if (ev) (void)hipEventRecord(ev[1], c.stream);
    if (e != hipSuccess) return e;
    hipStream_t ps = c.stream;
    if (overlap && c.n_sif > 0) {
        if ((e = hipEventRecord(c.ev_stp[b], c.stream)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c.side, c.ev_stp[b], 0)) != hipSuccess) return e;
        ps = c.side;
    }
    if (ev) (void)hipEventRecord(ev[2], ps);
    if (c.n_sif > 0) {
        const long nb2 = (c.n_sif + BLK - 1) / BLK;
        if (c.red)
            hipLaunchKernelGGL((k_phi_solid<L, T, true>), dim3(nb2), dim3(BLK), 0, ps, c.soff,
                               c.slinks, c.sdom, c.doms, (const T *)c.lq, c.phis, (long)c.n_sif, c.xpart, c.ndom,
                               args.evflag, args.evbatch, args.evidx, c.cfg.xcd_remap);
        else
            hipLaunchKernelGGL((k_phi_solid<L, T, false>), dim3(nb2), dim3(BLK), 0, ps, c.soff,
                               c.slinks, c.sdom, c.doms, (const T *)c.lq, c.phis, (long)c.n_sif, c.xpart, c.ndom,
                               args.evflag, args.evbatch, args.evidx, c.cfg.xcd_remap);
        e = hipGetLastError();
    }
    if (ev) (void)hipEventRecord(ev[3], ps);
    if (e == hipSuccess && ps != c.stream) {
        e = hipEventRecord(c.ev_phi[b], ps);
        c.phi_pending[b] = true;
        c.last_phi = b;
    }
    c.lq_next = 1 - b;
    c.cur = 1 - c.cur;
    c.phi_stale = true;
    return e;
}

hipError_t launch_step(Ctx &c, hipEvent_t *ev, bool overlap) {
    if (c.Q == 9) return c.fp64 ? step_impl<D2Q9, double>(c, ev, overlap) : step_impl<D2Q9, float>(c, ev, overlap);
    return c.fp64 ? step_impl<D3Q19, double>(c, ev, overlap) : step_impl<D3Q19, float>(c, ev, overlap);
}

hipError_t join_side(Ctx &c) {
    hipError_t e = hipSuccess;
    if (c.last_phi >= 0 && c.phi_pending[c.last_phi])
        e = hipStreamWaitEvent(c.stream, c.ev_phi[c.last_phi], 0);
    c.phi_pending[0] = c.phi_pending[1] = false;
    c.last_phi = -1;
    return e;
}

// working copies of the solid fraction <-> phi[] (site order)
__global__ __launch_bounds__(BLK) void k_phi_gather(long nf, const int32_t *__restrict__ nodeof,
                                                    long nsif, const int32_t *__restrict__ sif,
                                                    const double *__restrict__ phi,
                                                    double *__restrict__ phif, double *__restrict__ phis) {
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    if (t < nf) phif[t] = nodeof[t] >= 0 ? phi[nodeof[t]] : 0.0;
    if (t < nsif) phis[t] = phi[sif[t]];
}

__global__ __launch_bounds__(BLK) void k_phi_scatter(long nf, const int32_t *__restrict__ nodeof,
                                                     long nsif, const int32_t *__restrict__ sif,
                                                     const double *__restrict__ phif,
                                                     const double *__restrict__ phis,
                                                     double *__restrict__ phi) {
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    if (t < nf && nodeof[t] >= 0) phi[nodeof[t]] = phif[t];
    if (t < nsif) phi[sif[t]] = phis[t];
}

hipError_t launch_phi_gather(Ctx &c, long nf, long nsif) {
    const long n = nf > nsif ? nf : nsif;
    if (n > 0)
        hipLaunchKernelGGL(k_phi_gather, dim3((n + BLK - 1) / BLK), dim3(BLK), 0, c.stream, nf, c.nodeof,
                           nsif, c.sif, c.phi, c.phif, c.phis);
    c.phi_stale = false;
    c.full_check = true;   // values from outside the step: the next check scans them all
    return hipGetLastError();
}

hipError_t launch_phi_flush(Ctx &c) {
    if (!c.phi_stale) return hipSuccess;
    const long nf = c.n_slots, nsif = c.n_sif;
    const long n = nf > nsif ? nf : nsif;
    if (n > 0)
        hipLaunchKernelGGL(k_phi_scatter, dim3((n + BLK - 1) / BLK), dim3(BLK), 0, c.stream, nf, c.nodeof,
                           nsif, c.sif, c.phif, c.phis, c.phi);
    c.phi_stale = false;
    return hipGetLastError();
}

}  // namespace lbm
