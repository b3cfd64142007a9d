// lbm_events.hip -- phase change after a step (Sec. 2.4): a solid node whose
// solid fraction has fallen to 0 becomes fluid, a fluid node whose solid
// fraction has reached 1 becomes solid, and the geometry is rebuilt.
//
// Rules (the paper states them in words; the reading taken): a dissolving
// solid node (phi <= 0, at least one fluid neighbour) becomes fluid with C =
// mean C and rho = mean rho of its fluid neighbours and equilibrium
// populations at rest, and V_m C - phi is taken from the solid fraction of its
// solid neighbours in proportion to their rate constants (equal shares if all
// are 0; kept by the node itself if it has none); a precipitating fluid node
// (phi >= 1) adds V_m C to phi, passes phi - 1 in equal shares to its fluid
// neighbours (phi = 1) and drops its populations.  Both keep solute plus solid
// mass.  Events are taken in node order: a node pushed over its threshold by
// an earlier event of the same pass is taken in that pass if its index is
// larger, else at the next step.  Wall normals of solid nodes within two sites
// of a change are recomputed from the solid indicator.
//
// On the GPU: the step kernels flag a crossed threshold; a scan over all
// nodes then marks the candidates and the C and rho of every node are taken
// from the populations; one wavefront takes the events in node order (each
// lane reads and updates one neighbour; nodes that later events push over a
// threshold wait in an LDS bitmap window or a heap); then the wall normals
// near the changes are refreshed, the geometry (row words, tasks, links) is
// rebuilt in place and the populations are moved into the new compact
// layout.  The rule is serial in node order; the wavefront is used for the
// neighbourhood of one event at a time.
#include "lbm_internal.hpp"

namespace lbm {

constexpr uint32_t F_PEND = 1u << 29;  // geometry-flag bit: node waits in the heap
constexpr int EV_HEAP = 38912;         // pending nodes of one pass (LDS heap, 152 KiB)

struct EvRec {
    int64_t node;
    int32_t type;      // 0 dissolution, 1 precipitation
    int32_t pad;
    double C, rho;     // dissolution: the new node's concentration and density
};

template <class L>
__device__ __forceinline__ bool has_fluid_nb(const DomDev &D, long n, const uint8_t *solid) {
    int X, Y, Z;
    coords(D.box, n, &X, &Y, &Z);
    for (int i = 1; i < L::Q; i++) {
        int fc;
        const long y = site(D.box, X, Y, Z, L::ex[i], L::ey[i], L::ez[i], true, &fc);
        if (y >= 0 && !solid[y]) return true;
    }
    return false;
}

// candidates: solid with phi <= 0 and a fluid neighbour, fluid with phi >= 1
template <class L>
__global__ __launch_bounds__(BLK) void k_event_scan(const DomDev *doms, long N, const uint8_t *solid,
                                                    const double *phi, int32_t *cand, int32_t *any) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    int c = 0;
    if (solid[n]) c = phi[n] <= 0.0 && has_fluid_nb<L>(doms[0], n, solid);
    else c = phi[n] >= 1.0;
    cand[n] = c;
    if (c) atomicOr(any, 1);
}

__global__ __launch_bounds__(BLK) void k_event_list(long N, const int32_t *cand, const int32_t *pos,
                                                    int32_t *list, long cap) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N || !cand[n]) return;
    const long j = pos[n];
    if (j < cap) list[j] = (int32_t)n;
}

__global__ __launch_bounds__(BLK) void k_copy_i32(const int32_t *src, int32_t *dst, long n) {
    const long i = (long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// C and rho of the fluid node at compact index ko of the state before this
// pass (FP64 sums in direction order; the solute set is a compile-time mask,
// so all loads issue together)
template <class L, typename T, bool RED>
__device__ __forceinline__ void pop_moments(const DomDev &D, int ko, const T *f, const T *g, long S,
                                            double *C, double *rho) {
    constexpr uint32_t SM = sol_mask<L, RED>();
    double c = 0.0, r = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        r += (double)f[pidx(i, ko, L::Q)] + L::w[i] * D.rho0;
        if ((SM >> i) & 1u) c += (double)g[pidx(sol_slot(SM, i), ko, __builtin_popcount(SM))] + sol_w<L>(D, i) * D.c_ref;
    }
    *C = c;
    *rho = r;
}

// C and rho of every fluid node (dense, by node; 0 at solid nodes) from the
// populations before the pass, in parallel ahead of it: an event then reads
// its neighbours' moments in the same round as their state, instead of 2Q
// population loads behind a map lookup (populations do not change during the
// pass; a node that becomes fluid in it takes its moments from its record)
template <class L, typename T, bool RED>
__global__ __launch_bounds__(BLK) void k_event_moments(const DomDev *doms, long N, const int32_t *kof,
                                                       const T *f, const T *g, long S, double2 *mom) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    double C = 0.0, rho = 0.0;
    if (kof[n] >= 0) pop_moments<L, T, RED>(doms[0], kof[n], f, g, S, &C, &rho);
    mom[n] = make_double2(C, rho);
}

// moments of a node that became fluid earlier in this pass: equilibrium at
// rest of its record
template <class L>
__device__ __forceinline__ void rec_moments(const DomDev &D, const EvRec &e, double *C, double *rho) {
    double c = 0.0, r = 0.0;
    for (int i = 0; i < L::Q; i++) {
        r += L::w[i] * e.rho;
        c += D.ws[i] * e.C;   // 0 outside the solute set
    }
    *C = c;
    *rho = r;
}

// the same with the solute weights read from memory (ws: the domain's)
template <class L>
__device__ __forceinline__ void rec_moments_w(const double *ws, const EvRec &e, double *C, double *rho) {
    double c = 0.0, r = 0.0;
    for (int i = 0; i < L::Q; i++) {
        r += L::w[i] * e.rho;
        c += ws[i] * e.C;
    }
    *C = c;
    *rho = r;
}

// min-heap of the nodes that events push over a threshold during a pass
// (lane 0 only; in LDS)
__device__ __forceinline__ void heap_push(int32_t *h, int &n, int32_t v) {
    int i = n++;
    while (i > 0) {
        const int p = (i - 1) >> 1;
        if (h[p] <= v) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = v;
}

__device__ __forceinline__ int32_t heap_pop(int32_t *h, int &n) {
    const int32_t top = h[0];
    const int32_t last = h[--n];
    int i = 0;
    while (true) {
        const int l = 2 * i + 1;
        if (l >= n) break;
        const int r = l + 1;
        const int m = (r < n && h[r] < h[l]) ? r : l;
        if (h[m] >= last) break;
        h[i] = h[m];
        i = m;
    }
    if (n > 0) h[i] = last;
    return top;
}

// The pass for boxes less than 3 sites wide along some axis (a site can then
// be reached twice from one node, and lane 0 re-reads it after each update).
// One wavefront.  Lanes 1..Q-1 read, in parallel, the state of the neighbour
// along their direction (solid, phi, rate, marks, and its moments from the
// pass's moments or from its record if it became fluid earlier in the pass);
// lane 0 applies the rule and writes everything an event changes (solid, phi,
// kof_old, the records, the heap and its marks); the barrier at the end of
// every event makes those writes visible to the next event's reads.
// A node pushed over its threshold that is not a candidate of the pass goes
// into a min-heap (marked in the geometry flags, which the rebuild after the
// pass recomputes); the next node is the smaller of the list head and the
// heap top.  out[0] = events, out[1] = 1 if the records or the heap
// overflowed (the pass stops there).
template <class L, typename T, bool RED>
__global__ __launch_bounds__(64) void k_events(const DomDev *doms, const int32_t *list, long nlist,
                                               uint8_t *solid, double *phi, const double *kr,
                                               const int32_t *kof, int32_t *kof_old, const T *f,
                                               const T *g, long S, EvRec *rec, long cap,
                                               const int32_t *cand, uint32_t *gflags,
                                               const double2 *mom, int32_t *gheap, int32_t *out) {
    // the heap of pushed nodes and the next 64 list entries live in LDS; a
    // heap that outgrows the LDS moves to global memory (gheap, cap entries)
    __shared__ int32_t lheap[EV_HEAP];
    __shared__ int32_t lbuf[64];
    __shared__ int np_s, ne_s, ovf_s;
    __shared__ long cur_s, pos_s, lpos_s;
    const int lane = threadIdx.x;
    const DomDev D = doms[0];
    int32_t *heap = lheap;    // lane 0's view
    long hcap = cap < EV_HEAP ? cap : EV_HEAP;
    if (lane == 0) { np_s = 0; ne_s = 0; ovf_s = 0; pos_s = 0; }
    __syncthreads();
    long lchunk = -1;   // list position of lbuf[0]
    while (true) {
        const long pos = pos_s;
        if ((pos >> 6) != lchunk) {
            lchunk = pos >> 6;
            const long q = (lchunk << 6) + lane;
            lbuf[lane] = q < nlist ? list[q] : -1;
            __syncthreads();
        }
        if (lane == 0) {
            // next node: the smaller of the list head and the heap top (a
            // node is never in both); lpos_s: its list position, -1 if from
            // the heap
            long nxt = -1, lp = -1;
            const long a = pos < nlist ? (long)lbuf[pos & 63] : -1;
            const long b = np_s > 0 ? (long)heap[0] : -1;
            if (a >= 0 && (b < 0 || a < b)) {
                nxt = a;
                lp = pos;
                pos_s = pos + 1;
            } else if (b >= 0) {
                int np = np_s;
                nxt = heap_pop(heap, np);
                np_s = np;
            }
            if (ovf_s) nxt = -1;
            cur_s = nxt;
            lpos_s = lp;
        }
        __syncthreads();
        const long n = cur_s, lp = lpos_s;
        __syncthreads();
        if (n < 0) break;
        int X, Y, Z;
        coords(D.box, n, &X, &Y, &Z);
        // lanes 1..Q-1: the neighbour along their direction, its state as the
        // earlier events of the pass left it (lane 0's writes, visible after
        // the barrier) and its moments
        long y = -1;
        double Cy = 0.0, Ry = 0.0, Py = 0.0, Ky = 0.0;
        int fy = 0;   // bit 0 solid, bit 1 candidate of the pass, bit 2 in the heap
        if (lane >= 1 && lane < L::Q) {
            int fc;
            y = site(D.box, X, Y, Z, L::ex[lane], L::ey[lane], L::ez[lane], true, &fc);
            if (y >= 0) {
                fy = (solid[y] ? 1 : 0) | (cand[y] ? 2 : 0) | ((gflags[y] & F_PEND) ? 4 : 0);
                Py = phi[y];
                Ky = kr[y];
                // kof_old: the slot before the pass, or the record of a node
                // that became fluid in it
                const int ko = kof_old[y];
                const double2 m = mom[y];
                if (ko <= -2) {
                    rec_moments<L>(D, rec[-2 - ko], &Cy, &Ry);
                } else if (ko >= 0) {
                    Cy = m.x;
                    Ry = m.y;
                }
            }
        }
        // lane 0: the node's own state, read alongside its neighbours'
        bool sol_n = false;
        double phn = 0.0, Cx = 0.0, Rx = 0.0;
        if (lane == 0) {
            sol_n = solid[n] != 0;
            phn = phi[n];
            const int ko = kof_old[n];
            const double2 m = mom[n];
            if (!sol_n && phn >= 1.0) {
                if (ko >= 0) {
                    Cx = m.x;
                    Rx = m.y;
                } else {
                    rec_moments<L>(D, rec[-2 - ko], &Cx, &Rx);
                }
            }
        }
        long ys[L::Q];
        double cs[L::Q], rs[L::Q], ps[L::Q], ks[L::Q];
        int fs[L::Q];
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
            ys[i] = __shfl(y, i, 64);
            cs[i] = __shfl(Cy, i, 64);
            rs[i] = __shfl(Ry, i, 64);
            ps[i] = __shfl(Py, i, 64);
            ks[i] = __shfl(Ky, i, 64);
            fs[i] = __shfl(fy, i, 64);
        }
        if (lane == 0) {
            // on a box 3 or more sites wide along every axis the Q - 1
            // neighbours are distinct sites; otherwise a site may be reached
            // twice and its phi is read back after each update
            const bool distinct = D.box.nx >= 3 && D.box.ny >= 3 && (L::DIM == 2 || D.box.nz >= 3);
            auto push = [&](long v, bool pend) {
                if (distinct ? pend : (gflags[v] & F_PEND) != 0u) return;
                if (np_s >= hcap) {
                    if (heap != lheap || cap <= EV_HEAP) {
                        ovf_s = 1;
                        return;
                    }
                    for (int j = 0; j < np_s; j++) gheap[j] = lheap[j];
                    heap = gheap;
                    hcap = cap;
                }
                int np = np_s;
                heap_push(heap, np, (int32_t)v);
                np_s = np;
                gflags[v] |= F_PEND;
            };
            if (sol_n && phn <= 0.0) {
                double csum = 0.0, rsum = 0.0, wsum = 0.0;
                int nf = 0, nn = 0;
                for (int i = 1; i < L::Q; i++)
                    if (ys[i] >= 0 && !(fs[i] & 1)) { csum += cs[i]; rsum += rs[i]; nf++; }
                if (nf > 0) {
                    const double Cs = csum / nf, Rs = rsum / nf;
                    const double need = D.v_m * Cs - phn;
                    for (int i = 1; i < L::Q; i++)
                        if (ys[i] >= 0 && (fs[i] & 1)) { wsum += ks[i]; nn++; }
                    const int e = ne_s;
                    if (e >= cap) {
                        ovf_s = 1;
                    } else {
                        solid[n] = 0;
                        phi[n] = 0.0;
                        rec[e].node = n;
                        rec[e].type = 0;
                        rec[e].C = Cs;
                        rec[e].rho = Rs;
                        kof_old[n] = -2 - e;
                        ne_s = e + 1;
                        if (nn > 0) {
                            for (int i = 1; i < L::Q; i++) {
                                const long s = ys[i];
                                if (s < 0 || !(fs[i] & 1)) continue;
                                ps[i] = (distinct ? ps[i] : phi[s]) - need * (wsum > 0 ? ks[i] / wsum : 1.0 / nn);
                                phi[s] = ps[i];
                            }
                        } else {
                            phi[n] = 0.0 - need;
                        }
                        // later solid neighbours at or below zero now have a
                        // fluid neighbour: take them in this pass
                        for (int i = 1; i < L::Q; i++) {
                            const long s = ys[i];
                            if (s > n && !(fs[i] & 2) && (fs[i] & 1) && (distinct ? ps[i] : phi[s]) <= 0.0)
                                push(s, (fs[i] & 4) != 0);
                        }
                    }
                }
            } else if (!sol_n && phn >= 1.0) {
                const int e = ne_s;
                if (e >= cap) {
                    ovf_s = 1;
                } else {
                    const double phx = phn + D.v_m * Cx;
                    phi[n] = phx;
                    const double excess = phx - 1.0;
                    int nn = 0;
                    for (int i = 1; i < L::Q; i++)
                        if (ys[i] >= 0 && !(fs[i] & 1)) nn++;
                    if (nn > 0) {
                        for (int i = 1; i < L::Q; i++) {
                            const long s = ys[i];
                            if (s < 0 || (fs[i] & 1)) continue;
                            const double pnew = (distinct ? ps[i] : phi[s]) + excess / nn;
                            phi[s] = pnew;
                            if (s > n && !(fs[i] & 2) && pnew >= 1.0)
                                push(s, (fs[i] & 4) != 0);
                        }
                        phi[n] = 1.0;
                    }
                    solid[n] = 1;
                    rec[e].node = n;
                    rec[e].type = 1;
                    rec[e].C = Cx;
                    rec[e].rho = Rx;
                    ne_s = e + 1;
                }
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        out[0] = ne_s;
        out[1] = ovf_s;
    }
}

// The same pass with the work of an event spread over the lanes and no
// workgroup barrier, for boxes at least 3 sites wide along every axis (the
// Q - 1 neighbours of a node are then distinct sites).  The workgroup is one
// wavefront, whose memory operations complete in program order: a lane's
// read in a later event sees what any lane wrote in an earlier one, so the
// events need only compiler-level ordering between them.
//   Next node: the smallest of the list head, the far heap top and the first
// set bit of the pending window.  A node pushed less than EV_WIN sites past
// the current event goes into the window, a circular bitmap over node indices
// (every pending node lies within EV_WIN sites after the current one, so bit
// v mod EV_WIN names one node); a node pushed further goes into the far heap
// and is marked in the geometry flags.
//   An event: lanes 1..Q-1 read their neighbour's state and lane 0 the node's
// own in one round; each lane applies the rule's update to its neighbour
// (the shares are the same expressions as in the serial rule, so the values
// are identical); sums over the neighbours are taken in direction order.
constexpr int EV_WIN = 1 << 19;         // pending window (64 KiB bitmap)
constexpr int EV_WWORDS = EV_WIN / 64;
constexpr int EV_FHEAP = 16384;         // far heap entries in LDS (64 KiB)

__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double lane_d(double v, int l) {
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// first set position in [lo, hi) of the window (hi - lo <= EV_WIN), or -1.
// The word holding lo first, read by every lane alike (the next pending node
// is usually a few sites on); then 64 words at a time, one per lane.
__device__ __forceinline__ long window_first(const unsigned long long *bits, long lo, long hi, int lane) {
    const long w0 = lo & ~63L;
    {
        unsigned long long w = bits[(w0 >> 6) & (EV_WWORDS - 1)];
        w &= ~0ull << (lo - w0);
        if (hi - w0 < 64) w &= (1ull << (hi - w0)) - 1ull;
        const unsigned long long wu = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(w >> 32)) << 32) |
                                      (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)w);
        if (wu) return w0 + __builtin_ctzll(wu);
        if (hi <= w0 + 64) return -1;
    }
    for (long base = w0 + 64; base < hi; base += 64L * 64) {
        const long wp = base + 64L * lane;
        unsigned long long w = 0ull;
        if (wp < hi) {
            w = bits[(wp >> 6) & (EV_WWORDS - 1)];
            if (hi - wp < 64) w &= (1ull << (hi - wp)) - 1ull;
        }
        const unsigned long long m = __ballot(w != 0ull);
        if (m) {
            const int l = __builtin_ctzll(m);
            const unsigned long long wl = ((unsigned long long)__builtin_amdgcn_readlane((unsigned)(w >> 32), l) << 32) |
                                          (unsigned long long)__builtin_amdgcn_readlane((unsigned)w, l);
            return base + 64L * l + __builtin_ctzll(wl);
        }
    }
    return -1;
}

template <class L, typename T, bool RED>
__global__ __launch_bounds__(64) void k_events_wave(const DomDev *doms, const int32_t *list, long nlist,
                                                    uint8_t *solid, double *phi, const double *kr,
                                                    int32_t *kof_old, EvRec *rec, long cap,
                                                    const int32_t *cand, uint32_t *gflags,
                                                    const double2 *mom, int32_t *gheap, int32_t *out) {
    __shared__ unsigned long long bits[EV_WWORDS];
    __shared__ int32_t lheap[EV_FHEAP];
    __shared__ int32_t lbuf[64];
    const int lane = threadIdx.x;
    // only the box and V_m are kept in registers; the solute weights of a
    // record's moments are read from the domain record
    const Box bx = doms[0].box;
    const double v_m = doms[0].v_m;
    for (int w = lane; w < EV_WWORDS; w += 64) bits[w] = 0ull;
    wave_order();
    // wave-uniform selection state: list position and head a, far heap size
    // np, place (LDS or gheap) and top b, pending nodes in the window
    long pos = 0, apos = -1, lchunk = -1, nbits = 0, ne = 0, last = -1, a = LONG_MAX, b = LONG_MAX;
    int np = 0, inl = 1, ovf = 0;
    while (!ovf) {
        if (pos != apos) {
            apos = pos;
            if (pos < nlist && (pos >> 6) != lchunk) {
                lchunk = pos >> 6;
                const long q = (lchunk << 6) + lane;
                lbuf[lane] = q < nlist ? list[q] : -1;
                wave_order();
            }
            a = pos < nlist ? (long)lbuf[pos & 63] : LONG_MAX;
        }
        const long lim = a < b ? a : b;
        long c = -1;
        if (nbits > 0) {
            const long hi = last + 1 + EV_WIN - 1 < lim ? last + EV_WIN : lim;
            c = window_first(bits, last + 1, hi, lane);
        }
        long n;
        if (c >= 0) {
            n = c;
            if (lane == 0) atomicAnd(&bits[(c >> 6) & (EV_WWORDS - 1)], ~(1ull << (c & 63)));
            nbits--;
        } else if (a < b) {
            n = a;
            pos++;
        } else if (b != LONG_MAX) {
            n = b;
            int32_t top = 0;
            if (lane == 0) {
                int32_t *h = inl ? lheap : gheap;
                heap_pop(h, np);
                top = np > 0 ? h[0] : -1;
            }
            np = __builtin_amdgcn_readfirstlane(np);
            top = __builtin_amdgcn_readfirstlane(top);
            b = top >= 0 ? (long)top : LONG_MAX;
        } else {
            break;
        }
        wave_order();
        last = n;
        int X, Y, Z;
        coords(bx, n, &X, &Y, &Z);
        // lanes 1..Q-1: the neighbour along their direction; lane 0: the node.
        // Every lane loads from a valid node (its own or n), all in one round.
        long y = -1;
        if (lane >= 1 && lane < L::Q) {
            int fc;
            y = site(bx, X, Y, Z, L::ex[lane], L::ey[lane], L::ez[lane], true, &fc);
        }
        const bool have = lane == 0 || y >= 0;
        const long ya = y >= 0 ? y : n;
        const int sv = solid[ya];
        const int cv = cand[ya];
        const uint32_t gv = gflags[ya];
        const double pv = phi[ya], kv = kr[ya];
        const int ko = kof_old[ya];
        const double2 m = mom[ya];
        // bit 0 solid, bit 1 candidate of the pass, bit 2 in the far heap
        const int fy = have ? ((sv ? 1 : 0) | (lane > 0 && cv ? 2 : 0) | (lane > 0 && (gv & F_PEND) ? 4 : 0)) : 0;
        const double Py = have ? pv : 0.0, Ky = have ? kv : 0.0;
        // moments: from the populations before the pass, or from the record
        // of a node that became fluid in it
        double Cy = 0.0, Ry = 0.0;
        if (have && ko <= -2) {
            rec_moments_w<L>(doms[0].ws, rec[-2 - ko], &Cy, &Ry);
        } else if (have && ko >= 0) {
            Cy = m.x;
            Ry = m.y;
        }
        const bool sol_n = __builtin_amdgcn_readfirstlane(fy) & 1;
        const double phn = lane_d(Py, 0);
        const bool nb = lane >= 1 && y >= 0;
        const unsigned long long fm = __ballot(nb && !(fy & 1)), sm = __ballot(nb && (fy & 1));
        bool pushme = false;
        if (sol_n && phn <= 0.0) {
            const int nf = __builtin_popcountll(fm), nn = __builtin_popcountll(sm);
            if (nf > 0) {
                double csum = 0.0, rsum = 0.0, wsum = 0.0;
#pragma unroll
                for (int i = 1; i < L::Q; i++) {
                    if ((fm >> i) & 1ull) {
                        csum += lane_d(Cy, i);
                        rsum += lane_d(Ry, i);
                    }
                }
#pragma unroll
                for (int i = 1; i < L::Q; i++)
                    if ((sm >> i) & 1ull) wsum += lane_d(Ky, i);
                const double Cs = csum / nf, Rs = rsum / nf;
                const double need = v_m * Cs - phn;
                if (ne >= cap) {
                    ovf = 1;
                } else {
                    if (lane == 0) {
                        solid[n] = 0;
                        phi[n] = nn > 0 ? 0.0 : 0.0 - need;
                        rec[ne].node = n;
                        rec[ne].type = 0;
                        rec[ne].C = Cs;
                        rec[ne].rho = Rs;
                        kof_old[n] = (int32_t)(-2 - ne);
                    }
                    ne++;
                    if (nb && (fy & 1)) {
                        const double pn = Py - need * (wsum > 0 ? Ky / wsum : 1.0 / nn);
                        phi[y] = pn;
                        pushme = y > n && !(fy & 2) && pn <= 0.0;
                    }
                }
            }
        } else if (!sol_n && phn >= 1.0) {
            if (ne >= cap) {
                ovf = 1;
            } else {
                const double Cx = lane_d(Cy, 0), Rx = lane_d(Ry, 0);
                const double phx = phn + v_m * Cx;
                const double excess = phx - 1.0;
                const int nn = __builtin_popcountll(fm);
                if (nn > 0 && nb && !(fy & 1)) {
                    const double pn = Py + excess / nn;
                    phi[y] = pn;
                    pushme = y > n && !(fy & 2) && pn >= 1.0;
                }
                if (lane == 0) {
                    phi[n] = nn > 0 ? 1.0 : phx;
                    solid[n] = 1;
                    rec[ne].node = n;
                    rec[ne].type = 1;
                    rec[ne].C = Cx;
                    rec[ne].rho = Rx;
                }
                ne++;
            }
        }
        // pushes: near ones into the window, far ones into the heap
        pushme = pushme && !(fy & 4);
        const bool far = pushme && y - n >= EV_WIN;
        bool fresh = false;
        if (pushme && !far) {
            const unsigned long long bit = 1ull << (y & 63);
            const unsigned long long old = atomicOr(&bits[(y >> 6) & (EV_WWORDS - 1)], bit);
            fresh = !(old & bit);
        }
        nbits += __builtin_popcountll(__ballot(fresh));
        unsigned long long fmask = __ballot(far);
        if (fmask) {
            if (far) atomicOr(&gflags[y], F_PEND);
            int32_t top = 0;
            if (lane == 0) {
                while (fmask) {
                    const int l = __builtin_ctzll(fmask);
                    fmask &= fmask - 1ull;
                    const long v = (long)__builtin_amdgcn_readlane((unsigned)y, l);
                    const long hc = inl ? (cap < EV_FHEAP ? cap : EV_FHEAP) : cap;
                    if (np >= hc) {
                        if (!inl || cap <= EV_FHEAP) {
                            ovf = 1;
                            break;
                        }
                        for (int j = 0; j < np; j++) gheap[j] = lheap[j];
                        inl = 0;
                    }
                    heap_push(inl ? lheap : gheap, np, (int32_t)v);
                }
                top = np > 0 ? (inl ? lheap : gheap)[0] : -1;
            }
            np = __builtin_amdgcn_readfirstlane(np);
            inl = __builtin_amdgcn_readfirstlane(inl);
            ovf = __builtin_amdgcn_readfirstlane(ovf);
            top = __builtin_amdgcn_readfirstlane(top);
            b = top >= 0 ? (long)top : LONG_MAX;
        }
        wave_order();
    }
    if (lane == 0) {
        out[0] = (int32_t)ne;
        out[1] = ovf;
    }
}

// wall normals of solid nodes within two sites of every change (fluid view)
template <class L>
__global__ __launch_bounds__(BLK) void k_event_normals(const DomDev *doms, const EvRec *rec, long nev,
                                                       const uint8_t *solid, double *nrm) {
    constexpr int R = 2, SZ = 2 * R + 1;
    constexpr int NB = L::DIM == 3 ? SZ * SZ * SZ : SZ * SZ;
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    if (t >= nev * NB) return;
    const DomDev D = doms[0];
    const long e = t / NB;
    const int o = (int)(t - e * NB);
    const int dx = o % SZ - R, dy = (o / SZ) % SZ - R, dz = L::DIM == 3 ? o / (SZ * SZ) - R : 0;
    int X, Y, Z, fc;
    coords(D.box, rec[e].node, &X, &Y, &Z);
    const long s = site(D.box, X, Y, Z, dx, dy, dz, false, &fc);
    if (s < 0 || !solid[s]) return;
    int SX, SY, SZz;
    coords(D.box, s, &SX, &SY, &SZz);
    double gx = 0, gy = 0, gz = 0;
    for (int i = 1; i < L::Q; i++) {
        const long y = site(D.box, SX, SY, SZz, L::ex[i], L::ey[i], L::ez[i], false, &fc);
        const double ind = (y < 0 || solid[y]) ? 1.0 : 0.0;
        gx += L::w[i] * L::ex[i] * ind * 3.0;
        gy += L::w[i] * L::ey[i] * ind * 3.0;
        gz += L::w[i] * L::ez[i] * ind * 3.0;
    }
    const double m = sqrt(gx * gx + gy * gy + gz * gz);
    if (m > 0) { gx = -gx / m; gy = -gy / m; gz = -gz / m; }
    else { gx = gy = gz = 0.0; }
    nrm[3 * s] = gx;
    nrm[3 * s + 1] = gy;
    nrm[3 * s + 2] = gz;
}

// populations into the new compact layout: kept nodes move, a dissolved node
// starts at the equilibrium at rest of its event record
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_relayout(const DomDev *doms, long nf, const int32_t *nodeof,
                                                  const int32_t *kof_old, const EvRec *rec, long S,
                                                  const T *fo, const T *go, T *fn, T *gn) {
    const long k = (long)blockIdx.x * BLK + threadIdx.x;
    if (k >= nf) return;
    const DomDev D = doms[0];
    const long n = nodeof[k];
    if (n < 0) return;   // a hole
    const int ko = kof_old[n];
    if (ko >= 0) {
        const int qs = __builtin_popcount(D.smask);
        for (int i = 0; i < L::Q; i++) fn[pidx(i, k, L::Q)] = fo[pidx(i, ko, L::Q)];
        for (int s = 0; s < qs; s++) gn[pidx(s, k, qs)] = go[pidx(s, ko, qs)];
    } else {
        const EvRec &e = rec[-2 - ko];
        for (int i = 0; i < L::Q; i++) {
            fn[pidx(i, k, L::Q)] = (T)(L::w[i] * e.rho - L::w[i] * D.rho0);
            if ((D.smask >> i) & 1u)
                gn[pidx(sol_slot(D.smask, i), k, __builtin_popcount(D.smask))] = (T)(D.ws[i] * e.C - D.ws[i] * D.c_ref);
        }
    }
}

__global__ void k_zero2_i32(int32_t *p) {
    p[0] = 0;
    p[1] = 0;
}

// whether any node crossed a threshold: only the solid fraction of fluid
// nodes and of solid interface nodes changes in a step (the working copies,
// compact and solid-side order), and a solid node with a fluid neighbour is a
// solid interface node, so this covers every candidate of the full scan
__global__ __launch_bounds__(BLK) void k_event_check(long nf, const double *phif, long nsif,
                                                     const double *phis, int32_t *any) {
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    bool c = false;
    if (t < nf && phif[t] >= 1.0) c = true;
    if (t < nsif && phis[t] <= 0.0) c = true;
    if (__any(c) && (threadIdx.x & 63) == 0) atomicOr(any, 1);
}

template <class L, typename T>
static hipError_t events_impl(Ctx &c, bool flagged, int64_t *n_events, bool *overflow) {
    hipStream_t st = c.stream;
    const long N = c.N;
    const long nb = (N + BLK - 1) / BLK;
    *n_events = 0;
    *overflow = false;
    int32_t *any = c.iacc + 8, *cnt2 = c.iacc + 10;
    int32_t h[2] = {0, 0};
    hipError_t e = hipSuccess;
    if (!c.full_check) {
        // the step's kernels set the threshold flag if an interface node is
        // past its threshold (only interface nodes' solid fractions change in
        // a step, and every other node was checked when its value was last
        // set); the caller read it
        if (!flagged) return hipSuccess;
    } else {
        c.full_check = false;
        const long nf = c.n_slots, ns = c.n_sif, n = nf > ns ? nf : ns;
        hipLaunchKernelGGL(k_zero2_i32, dim3(1), dim3(1), 0, st, any);
        if (n > 0)
            hipLaunchKernelGGL(k_event_check, dim3((n + BLK - 1) / BLK), dim3(BLK), 0, st, nf, c.phif, ns,
                               c.phis, any);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h, any, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || h[0] == 0) return e;
    }
    // some node crossed: the site-ordered phi is brought up to date for the
    // full scan and the event pass
    if ((e = launch_phi_flush(c)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero2_i32, dim3(1), dim3(1), 0, st, any);
    hipLaunchKernelGGL((k_event_scan<L>), dim3(nb), dim3(BLK), 0, st, c.doms, N, c.solid, c.phi,
                       c.cnt, any);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, any, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess || h[0] == 0) return e;
    // candidates in node order
    if ((e = scan_excl(c, c.cnt, c.sidx, N, any + 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_event_list, dim3(nb), dim3(BLK), 0, st, N, c.cnt, c.sidx, c.evlist,
                       (long)c.ev_cap);
    hipLaunchKernelGGL(k_copy_i32, dim3(nb), dim3(BLK), 0, st, c.kof, c.kof_old, N);
    if ((e = hipMemcpyAsync(h, any + 1, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const long nlist = h[0] < c.ev_cap ? h[0] : c.ev_cap;
    if (h[0] > c.ev_cap) *overflow = true;
    double2 *mom = (double2 *)c.evmom;
    if (c.red)
        hipLaunchKernelGGL((k_event_moments<L, T, true>), dim3(nb), dim3(BLK), 0, st, c.doms, N, c.kof,
                           (const T *)c.f[c.cur], (const T *)c.g[c.cur], c.S, mom);
    else
        hipLaunchKernelGGL((k_event_moments<L, T, false>), dim3(nb), dim3(BLK), 0, st, c.doms, N, c.kof,
                           (const T *)c.f[c.cur], (const T *)c.g[c.cur], c.S, mom);
    const Box &bx = c.dom[0].box;
    const bool distinct = bx.nx >= 3 && bx.ny >= 3 && (L::DIM == 2 || bx.nz >= 3);
    if (distinct && c.red)
        hipLaunchKernelGGL((k_events_wave<L, T, true>), dim3(1), dim3(64), 0, st, c.doms, c.evlist, nlist,
                           c.solid, c.phi, c.kr, c.kof_old, (EvRec *)c.evrec, (long)c.ev_cap, c.cnt, c.flags,
                           mom, c.evheap, cnt2);
    else if (distinct)
        hipLaunchKernelGGL((k_events_wave<L, T, false>), dim3(1), dim3(64), 0, st, c.doms, c.evlist, nlist,
                           c.solid, c.phi, c.kr, c.kof_old, (EvRec *)c.evrec, (long)c.ev_cap, c.cnt, c.flags,
                           mom, c.evheap, cnt2);
    else if (c.red)
        hipLaunchKernelGGL((k_events<L, T, true>), dim3(1), dim3(64), 0, st, c.doms, c.evlist, nlist, c.solid,
                           c.phi, c.kr, c.kof, c.kof_old, (const T *)c.f[c.cur], (const T *)c.g[c.cur],
                           c.S, (EvRec *)c.evrec, (long)c.ev_cap, c.cnt, c.flags, mom, c.evheap, cnt2);
    else
        hipLaunchKernelGGL((k_events<L, T, false>), dim3(1), dim3(64), 0, st, c.doms, c.evlist, nlist, c.solid,
                           c.phi, c.kr, c.kof, c.kof_old, (const T *)c.f[c.cur], (const T *)c.g[c.cur],
                           c.S, (EvRec *)c.evrec, (long)c.ev_cap, c.cnt, c.flags, mom, c.evheap, cnt2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h, cnt2, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (h[1]) *overflow = true;
    *n_events = h[0];
    if (h[0] == 0) return hipSuccess;
    constexpr int NB = L::DIM == 3 ? 125 : 25;
    const long nt = (long)h[0] * NB;
    hipLaunchKernelGGL((k_event_normals<L>), dim3((nt + BLK - 1) / BLK), dim3(BLK), 0, st, c.doms,
                       (const EvRec *)c.evrec, (long)h[0], c.solid, c.nrm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipSuccess;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_zero_links(T *p, long n) {
    const long i = (long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <class L, typename T>
static hipError_t relayout_impl(Ctx &c) {
    const long nf = c.n_slots;
    // the last step's exchanges belong to the old link list
    if (c.n_links > 0)
        hipLaunchKernelGGL((k_zero_links<T>), dim3((c.n_links + BLK - 1) / BLK), dim3(BLK), 0,
                           c.stream, (T *)c.lq, (long)c.n_links);
    if (nf > 0)
        hipLaunchKernelGGL((k_relayout<L, T>), dim3((nf + BLK - 1) / BLK), dim3(BLK), 0, c.stream,
                           c.doms, nf, c.nodeof, c.kof_old, (const EvRec *)c.evrec, c.S,
                           (const T *)c.f[c.cur], (const T *)c.g[c.cur], (T *)c.f[1 - c.cur],
                           (T *)c.g[1 - c.cur]);
    c.cur = 1 - c.cur;
    return hipGetLastError();
}

hipError_t launch_events(Ctx &c, bool flagged, int64_t *n_events, bool *overflow) {
    if (c.Q == 9)
        return c.fp64 ? events_impl<D2Q9, double>(c, flagged, n_events, overflow)
                      : events_impl<D2Q9, float>(c, flagged, n_events, overflow);
    return c.fp64 ? events_impl<D3Q19, double>(c, flagged, n_events, overflow)
                  : events_impl<D3Q19, float>(c, flagged, n_events, overflow);
}

hipError_t launch_relayout(Ctx &c) {
    if (c.Q == 9) return c.fp64 ? relayout_impl<D2Q9, double>(c) : relayout_impl<D2Q9, float>(c);
    return c.fp64 ? relayout_impl<D3Q19, double>(c) : relayout_impl<D3Q19, float>(c);
}

size_t event_record_bytes() { return sizeof(EvRec); }

}  // namespace lbm
