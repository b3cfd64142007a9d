// lbm_geometry.hip -- geometry preparation (once per geometry, not per step).
//
// From the solid mask: node classes and reactive-link bits, the row words of
// the compact fluid layout, the compact <-> dense index maps, the wavefront
// tasks, the reactive-link list with beta = (1 - k_i)/(1 + k_i) per link
// (k_i of the selected scheme; a task's links form one range, by direction,
// then lane), and, per solid interface node, the list of its links in
// ascending direction order.
#include "lbm_internal.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// exclusive scan of int32 (in place allowed); total written to *total_dev
// ---------------------------------------------------------------------------
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = BLK * SCAN_PER;

__global__ __launch_bounds__(BLK) void k_scan_reduce(const int32_t *in, long n, int32_t *bsum) {
    const long base = (long)blockIdx.x * SCAN_TILE;
    long s = 0;
    for (int j = 0; j < SCAN_PER; j++) {
        const long i = base + (long)j * BLK + threadIdx.x;
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
    for (int j = 0; j < SCAN_PER; j++) {
        const long i = base + j;
        v[j] = i < n ? in[i] : 0;
        s += v[j];
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
    for (int j = 0; j < SCAN_PER; j++) {
        const long i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

__global__ void k_zero_total(int32_t *p) { *p = 0; }

hipError_t scan_excl(Ctx &c, const int32_t *in, int32_t *out, long n, int32_t *total_dev) {
    if (n <= 0) {
        // nothing to scan (a lattice without fluid nodes): the total is 0, and
        // no element of in, which the caller has not written, is read
        hipLaunchKernelGGL(k_zero_total, dim3(1), dim3(1), 0, c.stream, total_dev);
        return hipGetLastError();
    }
    const long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(BLK), 0, c.stream, in, n, c.bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, c.stream, c.bsum, nb, total_dev);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(BLK), 0, c.stream, in, out, n, c.bsum);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// node classes (every kernel below covers all domains of a batch; a thread
// finds its domain from the offset tables)
// ---------------------------------------------------------------------------
struct Geo {
    const DomDev *doms;
    const long *node_off, *word_off, *row_off;
    int ndom;
};

// domain d and local node index of global dense node n
__device__ __forceinline__ int dom_of(const Geo &g, long n, long *nl) {
    const int d = find_dom(g.node_off, g.ndom, n);
    *nl = n - g.doms[d].node_off;
    return d;
}

template <class L>
__global__ __launch_bounds__(BLK) void k_flags(Geo g, long N, const uint8_t *solid, uint32_t *flags,
                                               uint32_t *rmask) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        flags[n] = 0u;
        rmask[n] = 0u;
        return;
    }
    long nl;
    const int d = dom_of(g, n, &nl);
    const Box box = g.doms[d].box;
    const long base = g.doms[d].node_off;
    int X, Y, Z;
    coords(box, nl, &X, &Y, &Z);
    uint32_t fl = F_FLUID, rm = 0u;
    for (int i = 1; i < L::Q; i++) {
        int fc;
        const long y = site(box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], false, &fc);
        if (y < 0 || solid[base + y]) fl |= 1u << i;
        // a reactive link needs a direction of the solute set
        const long ys = site(box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], true, &fc);
        if (ys >= 0 && solid[base + ys] && ((g.doms[d].smask >> i) & 1u)) rm |= 1u << i;
    }
    if (rm) fl |= F_LINK;
    flags[n] = fl;
    rmask[n] = rm;
}

// one thread per row word: fluid mask of up to 64 nodes and its population count
__global__ __launch_bounds__(BLK) void k_row_words(Geo g, long RW, const uint8_t *solid,
                                                   RowWord *rows, int32_t *wcnt) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    if (j >= RW) return;
    const int d = find_dom(g.word_off, g.ndom, j);
    const DomDev &D = g.doms[d];
    const long jl = j - D.word_off;
    const long r = jl / D.W;
    const int w = (int)(jl - r * D.W);
    const long base = D.node_off + r * D.box.nx + 64L * w;
    const int len = min(64, D.box.nx - 64 * w);
    unsigned long long m = 0ull;
    for (int b = 0; b < len; b++)
        if (!solid[base + b]) m |= 1ull << b;
    rows[j].mask = m;
    rows[j].pad = 0;
    wcnt[j] = __popcll(m);
}

__global__ __launch_bounds__(BLK) void k_row_prefix(long RW, const int32_t *pre, RowWord *rows) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    if (j < RW) rows[j].pb = pre[j];
}

// dense <-> compact maps
__global__ __launch_bounds__(BLK) void k_compact(Geo g, long N, const uint8_t *solid,
                                                 const RowWord *rows, int32_t *nodeof, int32_t *kof) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        kof[n] = -1;
        return;
    }
    long nl;
    const int d = dom_of(g, n, &nl);
    const DomDev &D = g.doms[d];
    const long r = nl / D.box.nx;
    const int x = (int)(nl - r * D.box.nx);
    const RowWord w = rows[D.word_off + r * D.W + (x >> 6)];
    const int k = w.pb + __popcll(w.mask & ((1ull << (x & 63)) - 1ull));
    nodeof[k] = (int32_t)n;
    kof[n] = k;
}

__device__ __forceinline__ int row_fluid(const DomDev &D, const RowWord *rows, long r) {
    int c = 0;
    for (int w = 0; w < D.W; w++) c += __popcll(rows[D.word_off + r * D.W + w].mask);
    return c;
}

// Tasks.  A task is a run of at most 64 consecutive fluid nodes (compact
// order) whose pulls can be classified from a table of row words held one
// per lane: the rows y0 - 1 .. y0 + nr of the planes z - 1 .. z + 1 (one
// plane in 2D), words wlo .. wlo + nwd - 1 of each, at most 64 entries.
//  * Narrow rows (full rows fit for at least one task row, M >= 1): each
//    plane's fluid nodes cut into runs of 64 spanning at most M rows
//    (wlo = 0, nwd = W); a run that would need more rows ends early.
//  * Wide rows: runs stay within one row and cover a window of at most
//    maxw words (the words of x_first - 1 .. x_last + 1); a run whose nodes
//    would spread wider ends early.
template <class L>
__device__ __forceinline__ int task_max_rows(const DomDev &D) {
    const int per = 64 / D.W;                 // full table rows that fit
    const int m = (L::DIM == 3 ? per / 3 : per) - 2;
    return m > 255 ? 255 : m;                 // < 1: wide rows
}

template <class L>
__device__ __forceinline__ int task_max_words() {
    return 64 / (L::DIM == 3 ? 9 : 3);       // one task row: 3 (x 3) table rows
}

__device__ __forceinline__ void put_task(Task *tasks, int nt, long row, int k0, int cnt, int nr,
                                         int d, int wlo, int nwd, int ny) {
    Task t;
    t.row = (int32_t)row;
    t.k0 = k0;
    t.cnt = cnt | (nr << 8);
    t.dom = d;
    t.wlo = wlo;
    t.nwd = nwd;
    t.y0 = (int32_t)(row % ny);
    t.z = (int32_t)(row / ny);
    tasks[nt] = t;
}

// Task order.  In 3D the tasks are listed slab by slab: rows y in
// [s SL, (s + 1) SL) of every plane, planes in order, then the next slab.
// Consecutive tasks run on one XCD (the launch keeps runs of tiles
// together), so the tasks an XCD has in flight pull from a few planes of one
// slab, whose lines its L2 still holds from the neighbouring planes' tasks;
// in plane order the same reuse spans whole planes, more than the L2 keeps.
// A 2D lattice keeps row order (one slab).
template <class L>
__device__ __forceinline__ int slab_rows(const DomDev &D) {
    if (L::DIM == 2) return D.box.ny;
    const int s = 8192 / D.box.nx;            // about 32 rows of 256 nodes
    return s < 1 ? 1 : (s > D.box.ny ? D.box.ny : s);
}

// position of domain row r in the task order
template <class L>
__device__ __forceinline__ long row_pos(const DomDev &D, long r) {
    const int SL = slab_rows<L>(D), ny = D.box.ny;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const int sl = y / SL, h = min(SL, ny - sl * SL);
    return (long)sl * SL * D.box.nz + (long)z * h + (y - sl * SL);
}

// Walk rows ya .. yb - 1 of the plane starting at domain row r0 (y = 0);
// count the tasks, and write them when `tasks` is given (narrow rows).
template <class L>
__device__ int plane_tasks(const DomDev &D, int d, const RowWord *rows, long r0, int ya, int yb,
                           Task *tasks) {
    const int M = task_max_rows<L>(D);
    int nt = 0;
    int count = 0, srow = 0, sk = 0;   // the open run: nodes, first row, first node
    auto emit = [&](int last_row) {
        if (count == 0) return;
        if (tasks) put_task(tasks, nt, r0 + srow, sk, count, last_row - srow + 1, d, 0, D.W, D.box.ny);
        nt++;
        count = 0;
    };
    int last = ya;
    for (int y = ya; y < yb; y++) {
        const long r = r0 + y;
        int c = row_fluid(D, rows, r);
        if (c == 0) continue;
        int k = rows[D.word_off + r * D.W].pb;
        if (count > 0 && y - srow + 1 > M) emit(last);
        while (c > 0) {
            if (count == 0) {
                srow = y;
                sk = k;
            }
            const int take = min(c, 64 - count);
            count += take;
            c -= take;
            k += take;
            last = y;
            if (count == 64) emit(y);
        }
    }
    emit(last);
    return nt;
}

// Tasks of one wide row r (count; write when `tasks` is given).  A task that
// ends short of 64 nodes ends at a word boundary: the window is checked once
// per word, for all of the word's nodes (a full task may end inside a word).
template <class L>
__device__ int wide_row_tasks(const DomDev &D, int d, const RowWord *rows, long r, Task *tasks) {
    const int W = D.W, maxw = task_max_words<L>();
    int nt = 0, count = 0, k0 = 0, wlo = 0, whi = 0;
    auto emit = [&]() {
        if (count == 0) return;
        if (tasks) put_task(tasks, nt, r, k0, count, 1, d, wlo, whi - wlo + 1, D.box.ny);
        nt++;
        count = 0;
    };
    for (int w = 0; w < W; w++) {
        const RowWord rw = rows[D.word_off + r * W + w];
        unsigned long long m = rw.mask;
        int k = rw.pb;
        if (m && count > 0) {
            const int xl = 64 * w + 63 - __clzll((long long)m);
            if (min(W - 1, (xl + 1) >> 6) - wlo + 1 > maxw) emit();
        }
        while (m) {
            const int x = 64 * w + __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const int hi = min(W - 1, (x + 1) >> 6);
            if (count == 64) emit();
            if (count == 0) {
                k0 = k;
                wlo = x == 0 ? 0 : (x - 1) >> 6;
            }
            whi = hi;
            count++;
            k++;
        }
    }
    emit();
    return nt;
}

template <class L>
__global__ __launch_bounds__(BLK) void k_row_ntasks(Geo g, long R, const RowWord *rows, int32_t *nt) {
    const long rg = (long)blockIdx.x * BLK + threadIdx.x;
    if (rg >= R) return;
    const int d = find_dom(g.row_off, g.ndom, rg);
    const DomDev &D = g.doms[d];
    const long r = rg - D.row_off;
    const long pos = D.row_off + row_pos<L>(D, r);
    if (task_max_rows<L>(D) >= 1) {
        // the first row of each slab segment of a plane walks the segment
        const int SL = slab_rows<L>(D), y = (int)(r % D.box.ny);
        nt[pos] = y % SL == 0 ? plane_tasks<L>(D, d, rows, r - y, y, min(y + SL, D.box.ny), nullptr) : 0;
    } else {
        nt[pos] = wide_row_tasks<L>(D, d, rows, r, nullptr);
    }
}

template <class L>
__global__ __launch_bounds__(BLK) void k_row_tasks(Geo g, long R, const RowWord *rows,
                                                   const int32_t *tbase, Task *tasks) {
    const long rg = (long)blockIdx.x * BLK + threadIdx.x;
    if (rg >= R) return;
    const int d = find_dom(g.row_off, g.ndom, rg);
    const DomDev &D = g.doms[d];
    const long r = rg - D.row_off;
    const long pos = D.row_off + row_pos<L>(D, r);
    if (task_max_rows<L>(D) >= 1) {
        const int SL = slab_rows<L>(D), y = (int)(r % D.box.ny);
        if (y % SL == 0) plane_tasks<L>(D, d, rows, r - y, y, min(y + SL, D.box.ny), tasks + tbase[pos]);
    } else {
        wide_row_tasks<L>(D, d, rows, r, tasks + tbase[pos]);
    }
}

// ---------------------------------------------------------------------------
// Slots.  Every task gets a block of 64 population slots of its own, the
// blocks in node order: the nodes of the task of rank r (in node order) take
// slots 64 r .. 64 r + cnt - 1, so that a wavefront's own loads and stores
// cover whole 256-byte lines of the blocked population arrays.  A task that
// ends short of 64 nodes ends at a row-word boundary (a full one may end
// inside a word, and then its successor's slots follow on without a gap), so
// the nodes of every row word still have consecutive slots: the row word's pb
// becomes the slot of its first fluid node.  Slots past a short task's nodes
// are holes (nodeof = -1) that no kernel reads or writes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLK) void k_task_marks(const Task *tasks, long nt, int32_t *mark) {
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    if (t < nt) mark[tasks[t].k0] = 1;
}

// tasks: compact k0 -> 64 * rank; tstart[rank] = the compact k0
__global__ __launch_bounds__(BLK) void k_task_slots(Task *tasks, long nt, const int32_t *rank,
                                                    int32_t *tstart) {
    const long t = (long)blockIdx.x * BLK + threadIdx.x;
    if (t >= nt) return;
    const int k0 = tasks[t].k0, r = rank[k0];
    tstart[r] = k0;
    tasks[t].k0 = 64 * r;
}

// slot of compact index c (rank: exclusive scan of the task-start marks)
__device__ __forceinline__ int slot_of(int c, const int32_t *mark, const int32_t *rank,
                                       const int32_t *tstart) {
    const int r = rank[c] + mark[c] - 1;
    return 64 * r + (c - tstart[r]);
}

__global__ __launch_bounds__(BLK) void k_slot_nodes(long N, int32_t *kof, int32_t *nodeof,
                                                    const int32_t *mark, const int32_t *rank,
                                                    const int32_t *tstart) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N || kof[n] < 0) return;
    const int s = slot_of(kof[n], mark, rank, tstart);
    kof[n] = s;
    nodeof[s] = (int32_t)n;
}

// every word, empty ones too: a word's pb is the slot of the first fluid node
// at or after it (the kernels find a lane's row by comparing its slot with the
// pb of each row's first word), ns past the last one
__global__ __launch_bounds__(BLK) void k_slot_words(long RW, RowWord *rows, long nf, long ns,
                                                    const int32_t *mark, const int32_t *rank,
                                                    const int32_t *tstart) {
    const long j = (long)blockIdx.x * BLK + threadIdx.x;
    if (j >= RW) return;
    const int c = rows[j].pb;
    rows[j].pb = c < nf ? slot_of(c, mark, rank, tstart) : (int32_t)ns;
}

__global__ void k_fill_i32(int32_t *p, long n, int32_t v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// reactive links per slot (holes have none), then the link records
__global__ __launch_bounds__(BLK) void k_link_count(long ns, const int32_t *nodeof,
                                                    const uint32_t *rmask, int32_t *cnt) {
    const long k = (long)blockIdx.x * BLK + threadIdx.x;
    if (k < ns) cnt[k] = nodeof[k] >= 0 ? __popc(rmask[nodeof[k]]) : 0;
}

// Link order.  The links of a task's nodes occupy one range (from lbase of
// its first node); within it they are ordered by direction, then by node, so
// that the lanes of a wavefront holding a link along the same direction read
// its coefficient and write its exchange at consecutive addresses.  The link
// records are written in that order, one wavefront per task (lanes = the
// task's nodes): a link's index is the task's base, the links of the earlier
// directions and the lanes below holding the same direction (the fused step's
// numbering).
template <class L, typename T>
__global__ __launch_bounds__(BLK) void k_links(Geo g, const Task *tasks, long ntasks, const int32_t *nodeof,
                                               const uint32_t *rmask, const int32_t *lbase,
                                               const double *nrm, const double *kr, T *lbeta,
                                               int32_t *lnode, int32_t *lsolid, uint8_t *ldir,
                                               const double *ceq, T *lceq) {
    const long t = (long)blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
    if (t >= ntasks) return;
    const int lane = threadIdx.x & 63;
    const Task tk = tasks[t];
    const int cnt = tk.cnt & 255;
    const bool active = lane < cnt;
    const int k = tk.k0 + (active ? lane : 0);
    const long n = nodeof[k];
    const uint32_t rm = active ? rmask[n] : 0u;
    const int base = __shfl(lbase[k], 0, 64);   // the task's first link
    const unsigned long long below = (1ull << lane) - 1ull;
    long nl;
    const int d = dom_of(g, n, &nl);
    const DomDev &D = g.doms[d];
    int X, Y, Z;
    coords(D.box, nl, &X, &Y, &Z);
    int off = 0;
    for (int i = 1; i < L::Q; i++) {
        const bool has = (rm >> i) & 1u;
        const unsigned long long bal = __ballot(has);
        if (has) {
            const int l = base + off + __popcll(bal & below);
            int fc;
            const long s = D.node_off + site(D.box, X, Y, Z, -L::ex[i], -L::ey[i], -L::ez[i], true, &fc);
            const double en = L::ex[i] * nrm[3 * s] + L::ey[i] * nrm[3 * s + 1] + L::ez[i] * nrm[3 * s + 2];
            const double kv = kr[s];
            double kap;
            if (D.scheme == LBM_SV) kap = en > 0 ? kv * en / D.cs2s : 0.0;
            else if (D.scheme == LBM_SPJ) kap = en > 0 ? D.gamma * kv / (D.cs2s * en) : 0.0;
            else kap = en > 0 ? D.gamma * kv * en / D.cs2s : 0.0;
            // pre-collision source with both neighbours solid: fall back to the
            // node's own post-collision population, whose effective rate is gamma k
            if (D.mech == LBM_PRECOLL && (rm & (1u << L::opp[i]))) kap = kap / D.gamma;
            // anti-bounce-back (the k -> infinity limit) at reactive solid nodes;
            // a solid node with k_r = 0 keeps plain bounce-back (kap = 0)
            const double beta = (D.scheme == LBM_ABB && kv > 0.0) ? -1.0 : (1.0 - kap) / (1.0 + kap);
            lbeta[l] = (T)beta;
            // per-node C_eq (deviation form); the uniform value until one is given
            if (lceq) lceq[l] = (T)((ceq ? ceq[s] : D.ceq_dev + D.c_ref) - D.c_ref);
            lnode[l] = (int32_t)n;
            lsolid[l] = (int32_t)s;
            ldir[l] = (uint8_t)i;
        }
        off += __popcll(bal);
    }
}

// Solid side of the link list, built from the links themselves: link l joins
// fluid node lnode[l] to solid node lsolid[l] along direction ldir[l], and a
// solid node has at most one link per direction, so the set of directions of
// its links (a bit mask) gives both its link count and each link's rank in
// direction order.
__global__ __launch_bounds__(BLK) void k_solid_dirs(long nl, const int32_t *lsolid, const uint8_t *ldir,
                                                    uint32_t *smask) {
    const long l = (long)blockIdx.x * BLK + threadIdx.x;
    if (l < nl) atomicOr(&smask[lsolid[l]], 1u << ldir[l]);
}

__global__ __launch_bounds__(BLK) void k_solid_mark(long N, const uint32_t *smask, int32_t *ind) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n < N) ind[n] = smask[n] != 0u ? 1 : 0;
}

// per solid interface node (position idx[n] in node order): its node, link
// count (scanned into offsets afterwards) and domain
__global__ __launch_bounds__(BLK) void k_solid_nodes(Geo g, long N, const uint32_t *smask, const int32_t *idx,
                                                     int32_t *sif, int32_t *soff, int32_t *sdom) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    const uint32_t m = smask[n];
    if (!m) return;
    long nl;
    const int j = idx[n];
    sif[j] = (int32_t)n;
    soff[j] = __popc(m);
    sdom[j] = dom_of(g, n, &nl);
}

// each link into its solid node's segment, in direction order
__global__ __launch_bounds__(BLK) void k_solid_links(long nl, const int32_t *lsolid, const uint8_t *ldir,
                                                     const uint32_t *smask, const int32_t *idx,
                                                     const int32_t *soff, int32_t *slinks) {
    const long l = (long)blockIdx.x * BLK + threadIdx.x;
    if (l >= nl) return;
    const int32_t s = lsolid[l];
    const uint32_t m = smask[s];
    slinks[soff[idx[s]] + __popc(m & ((1u << ldir[l]) - 1u))] = (int32_t)l;
}

// lattice-gradient normal of the solid indicator (used when no normals are given)
template <class L>
__global__ __launch_bounds__(BLK) void k_fd_normals(Geo g, long N, const uint8_t *solid, double *nrm) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    double gx = 0, gy = 0, gz = 0;
    if (solid[n]) {
        long nl;
        const int d = dom_of(g, n, &nl);
        const DomDev &D = g.doms[d];
        int X, Y, Z;
        coords(D.box, nl, &X, &Y, &Z);
        for (int i = 1; i < L::Q; i++) {
            int fc;
            const long y = site(D.box, X, Y, Z, L::ex[i], L::ey[i], L::ez[i], false, &fc);
            const double ind = (y < 0 || solid[D.node_off + y]) ? 1.0 : 0.0;
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

__global__ __launch_bounds__(BLK) void k_node_defaults(Geo g, long N, const uint8_t *solid,
                                                       const double *kr_in, const double *phi_in,
                                                       double *kr, double *phi) {
    const long n = (long)blockIdx.x * BLK + threadIdx.x;
    if (n >= N) return;
    long nl;
    const int d = dom_of(g, n, &nl);
    kr[n] = kr_in ? kr_in[n] : g.doms[d].kr0;
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

// fluid interface nodes (at least one reactive link): indicator for a scan
__global__ __launch_bounds__(BLK) void k_iface_mark(long nf, const int32_t *lcnt, int32_t *ind) {
    const long k = (long)blockIdx.x * BLK + threadIdx.x;
    if (k < nf) ind[k] = lcnt[k] > 0 ? 1 : 0;
}

static hipError_t read_ints(Ctx &c, const int32_t *dev, int32_t *host, int n) {
    hipError_t e = hipMemcpyAsync(host, dev, n * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c.stream);
}

template <class L, typename T>
static hipError_t geometry_impl(Ctx &c, const uint8_t *solid, const double *normals,
                                const double *k_r, const double *phi0, int64_t *n_links,
                                int64_t *n_sif) {
    const long N = c.N, R = c.R, RW = c.RW;
    const long nb = (N + BLK - 1) / BLK;
    auto blocks = [](long n) { return dim3((unsigned)((n + BLK - 1) / BLK)); };
    hipStream_t st = c.stream;
    Geo g;
    g.doms = c.doms;
    g.node_off = c.dnode_off;
    g.word_off = c.dword_off;
    g.row_off = c.drow_off;
    g.ndom = c.ndom;
    hipError_t e;
    hipLaunchKernelGGL(k_copy_solid, dim3(nb), dim3(BLK), 0, st, N, solid, c.solid);
    hipLaunchKernelGGL(k_node_defaults, dim3(nb), dim3(BLK), 0, st, g, N, c.solid, k_r, phi0, c.kr,
                       c.phi);
    if (normals) {
        if (normals != c.nrm) {
            e = hipMemcpyAsync(c.nrm, normals, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
    } else {
        hipLaunchKernelGGL((k_fd_normals<L>), dim3(nb), dim3(BLK), 0, st, g, N, c.solid, c.nrm);
    }
    hipLaunchKernelGGL((k_flags<L>), dim3(nb), dim3(BLK), 0, st, g, N, c.solid, c.flags, c.rmask);
    // row words and compact maps
    hipLaunchKernelGGL(k_row_words, blocks(RW), dim3(BLK), 0, st, g, RW, c.solid, c.rows, c.cnt);
    if ((e = scan_excl(c, c.cnt, c.sidx, RW, c.iacc)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_prefix, blocks(RW), dim3(BLK), 0, st, RW, c.sidx, c.rows);
    hipLaunchKernelGGL(k_compact, dim3(nb), dim3(BLK), 0, st, g, N, c.solid, c.rows, c.nodeof, c.kof);
    int32_t nf = 0;
    if ((e = read_ints(c, c.iacc, &nf, 1)) != hipSuccess) return e;
    c.n_fluid = nf;
    // wavefront tasks
    hipLaunchKernelGGL((k_row_ntasks<L>), blocks(R), dim3(BLK), 0, st, g, R, c.rows, c.cnt);
    if ((e = scan_excl(c, c.cnt, c.sidx, R, c.iacc)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_row_tasks<L>), blocks(R), dim3(BLK), 0, st, g, R, c.rows, c.sidx, c.tasks);
    int32_t nt = 0;
    if ((e = read_ints(c, c.iacc, &nt, 1)) != hipSuccess) return e;
    c.n_tasks = nt;
    // slots: a 64-aligned block per task when they fit the arrays, else the
    // compact indices themselves
    long ns = nf;
    if (nt > 0 && 64L * nt <= c.S) {
        ns = 64L * nt;
        const long nfl0 = nf > 0 ? nf : 1;
        hipLaunchKernelGGL(k_fill_i32, blocks(nfl0), dim3(BLK), 0, st, c.cnt, (long)nf, 0);
        hipLaunchKernelGGL(k_task_marks, blocks(nt), dim3(BLK), 0, st, c.tasks, (long)nt, c.cnt);
        if ((e = scan_excl(c, c.cnt, c.sidx, nf, c.iacc)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_task_slots, blocks(nt), dim3(BLK), 0, st, c.tasks, (long)nt, c.sidx, c.lbase);
        hipLaunchKernelGGL(k_fill_i32, blocks(ns), dim3(BLK), 0, st, c.nodeof, ns, -1);
        hipLaunchKernelGGL(k_slot_nodes, dim3(nb), dim3(BLK), 0, st, N, c.kof, c.nodeof, c.cnt, c.sidx,
                           c.lbase);
        hipLaunchKernelGGL(k_slot_words, blocks(RW), dim3(BLK), 0, st, RW, c.rows, (long)nf, ns, c.cnt,
                           c.sidx, c.lbase);
    }
    c.n_slots = ns;
    // reactive links
    const long nfl = ns > 0 ? ns : 1;
    hipLaunchKernelGGL(k_link_count, blocks(nfl), dim3(BLK), 0, st, ns, c.nodeof, c.rmask, c.cnt);
    if ((e = scan_excl(c, c.cnt, c.lbase, ns, c.iacc)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_iface_mark, blocks(nfl), dim3(BLK), 0, st, ns, c.cnt, c.sidx);
    if ((e = scan_excl(c, c.sidx, c.sidx, ns, c.iacc + 2)) != hipSuccess) return e;
    int32_t t4[4] = {0, 0, 0, 0};
    if ((e = read_ints(c, c.iacc, t4, 4)) != hipSuccess) return e;
    const int32_t tot = t4[0];
    c.n_fluid_iface = t4[2];
    *n_links = tot;
    if (tot > c.max_links) return hipSuccess;  // the caller reports the capacity error
    if (c.n_tasks > 0)
        hipLaunchKernelGGL((k_links<L, T>), dim3((c.n_tasks + BLK / 64 - 1) / (BLK / 64)), dim3(BLK), 0, st, g,
                           c.tasks, (long)c.n_tasks, c.nodeof, c.rmask, c.lbase, c.nrm, c.kr, (T *)c.lbeta,
                           c.lnode, c.lsolid, c.ldir, c.ceq_set ? c.ceq : nullptr, (T *)c.lceq);
    // solid side: per solid interface node, its links in direction order
    uint32_t *smask = (uint32_t *)c.cnt;
    hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(BLK), 0, st, c.cnt, N, 0);
    if (tot > 0)
        hipLaunchKernelGGL(k_solid_dirs, blocks(tot), dim3(BLK), 0, st, (long)tot, c.lsolid, c.ldir, smask);
    hipLaunchKernelGGL(k_solid_mark, dim3(nb), dim3(BLK), 0, st, N, smask, c.sidx);
    if ((e = scan_excl(c, c.sidx, c.sidx, N, c.iacc)) != hipSuccess) return e;
    int32_t t2[2] = {0, 0};
    if ((e = read_ints(c, c.iacc, t2, 1)) != hipSuccess) return e;
    *n_sif = t2[0];
    hipLaunchKernelGGL(k_solid_nodes, dim3(nb), dim3(BLK), 0, st, g, N, smask, c.sidx, c.sif, c.soff, c.sdom);
    if ((e = scan_excl(c, c.soff, c.soff, t2[0], c.iacc + 1)) != hipSuccess) return e;
    if (tot > 0)
        hipLaunchKernelGGL(k_solid_links, blocks(tot), dim3(BLK), 0, st, (long)tot, c.lsolid, c.ldir, smask,
                           c.sidx, c.soff, c.slinks);
    if ((e = read_ints(c, c.iacc + 1, t2 + 1, 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, c.soff, (long)t2[0], t2[1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (t2[1] != tot) return hipErrorUnknown;  // every link has exactly one solid end
    if ((e = launch_phi_gather(c, ns, t2[0])) != hipSuccess) return e;
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

}  // namespace lbm
