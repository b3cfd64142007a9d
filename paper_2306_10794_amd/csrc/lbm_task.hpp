// lbm_task.hpp -- neighbour classification of one task (up to 64 consecutive
// fluid nodes of one x-row, one per lane), shared by the step kernels and the
// adjoint kernels.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

// Compact index of the fluid site (xx, yy, zz) (fluid view of the box), -1 if
// that site is solid, -2 if it is outside a non-periodic face.
__device__ __forceinline__ int nb_compact(const RowWord *__restrict__ rows, int W, const Box &b,
                                          int xx, int yy, int zz) {
    int fc;
    if (!wrap_site(b, xx, yy, zz, &fc)) return -2;
    const RowWord w = rows[(long)(yy + b.ny * zz) * W + (xx >> 6)];
    const unsigned long long bit = 1ull << (xx & 63);
    if (!(w.mask & bit)) return -1;
    return w.pb + __popcll(w.mask & (bit - 1ull));
}

// The row words of every row a task pulls from: a table of the rows
// y0 - 1 .. y0 + nr of the planes z - 1 .. z + 1 (one plane in 2D) for a task
// of nr rows from (y0, z); lane j holds word (j % W) of table row (j / W);
// other lanes read them with cross-lane shuffles.
struct RowSlots {
    unsigned long long wm;
    int wpb;
    int TY;       // table rows per plane, nr + 2
    int wlo, nwd; // window of words of each table row
    bool fit;     // the table fits the 64 lanes
};

template <class L>
__device__ __forceinline__ RowSlots load_row_slots(const RowWord *__restrict__ rows, const Box &b,
                                                   int W, int lane, int y0, int z, int nr, int wlo,
                                                   int nwd) {
    RowSlots rs;
    rs.TY = nr + 2;
    rs.wlo = wlo;
    rs.nwd = nwd;
    const int NSL = (L::DIM == 3 ? 3 : 1) * rs.TY;
    rs.fit = NSL * nwd <= 64;
    rs.wm = 0ull;
    rs.wpb = 0;
    if (rs.fit && lane < NSL * nwd) {
        const int sl = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)nwd));
        const int w = wlo + (lane - sl * nwd);
        const int sq = (int)(((float)sl + 0.5f) * __builtin_amdgcn_rcpf((float)rs.TY));
        int yy = y0 - 1 + (sl - sq * rs.TY), zz = L::DIM == 3 ? z - 1 + sq : z, xx = 0, fc;
        if (wrap_site(b, xx, yy, zz, &fc)) {
            const RowWord rw = rows[(long)(yy + b.ny * zz) * W + w];
            rs.wm = rw.mask;
            rs.wpb = rw.pb;
        }
    }
    return rs;
}

// row of the task (0 .. nr - 1) that compact index k lies in
template <class L>
__device__ __forceinline__ int task_row(const RowSlots &rs, int W, int nr, int k) {
    int ry = 0;
    for (int j = 1; j < nr; j++) {
        const int pbj = __shfl(rs.wpb, ((L::DIM == 3 ? rs.TY : 0) + j + 1) * rs.nwd, 64);
        if (k >= pbj) ry = j;
    }
    return ry;
}

// Upstream neighbour x - e_i of node (x, y, z) (compact index k) for every i:
// kk[i] = its compact index, -1 if solid, -2 if outside a non-periodic face
// (fluid view).  solidnb: bits of solid upstream neighbours; cross / cross_hi:
// bits whose upstream site lies beyond the low or high face of the inlet axis
// (cross_hi: the high one).  Every lane of the wavefront must call it (the
// shuffles read zero from inactive lanes).
template <class L>
__device__ __forceinline__ void classify(const RowWord *__restrict__ rows, const Box &b, int W,
                                         const RowSlots &rs, int ry, int x, int y, int z, int k, int *kk,
                                         uint32_t &solidnb, uint32_t &cross, uint32_t &cross_hi) {
    // the faces the node lies on give the directions whose pull leaves the
    // box, crosses the inlet or outlet plane, or wraps with a row shift
    constexpr uint32_t PX = dir_mask<L>(0, 1), NX = dir_mask<L>(0, -1);
    constexpr uint32_t PY = dir_mask<L>(1, 1), NY = dir_mask<L>(1, -1);
    constexpr uint32_t PZ = dir_mask<L>(2, 1), NZ = dir_mask<L>(2, -1);
    const uint32_t fx = (x == 0 ? PX : 0u) | (x == b.nx - 1 ? NX : 0u);
    const uint32_t fy = (y == 0 ? PY : 0u) | (y == b.ny - 1 ? NY : 0u);
    const uint32_t fz = (z == 0 ? PZ : 0u) | (z == b.nz - 1 ? NZ : 0u);
    const uint32_t outm = (b.per[0] ? 0u : fx) | (b.per[1] ? 0u : fy) | (b.per[2] ? 0u : fz);
    const uint32_t shiftm = (b.per[0] && b.shift != 0) ? fx : 0u;
    const int ax = b.inlet_axis;
    cross = 0u;
    cross_hi = 0u;
    if (ax >= 0) {
        const uint32_t f = ax == 0 ? fx : (ax == 1 ? fy : fz);
        cross = f;
        cross_hi = f & ~(ax == 0 ? PX : (ax == 1 ? PY : PZ));
    }
    // the three x offsets x + 1, x, x - 1 (e_x = -1, 0, 1): table column (-1:
    // outside the table) and bit within the row word
    int tcol[3];
    unsigned long long tbit[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        const int xn = x + 1 - v;
        const int xw = !b.per[0] ? xn : (xn < 0 ? xn + b.nx : (xn >= b.nx ? xn - b.nx : xn));
        const int xs = min(max(xw, 0), b.nx - 1);
        const int tw = (xs >> 6) - rs.wlo;
        tcol[v] = (rs.fit && tw >= 0 && tw < rs.nwd) ? ry * rs.nwd + tw : -1;
        tbit[v] = 1ull << (xs & 63);
    }
    solidnb = 0u;
    kk[0] = k;
    // every pull of every lane resolved by the table (decided once per
    // wavefront): straight-line selects, as in the fused step
    const bool tab_ok = rs.fit && outm == 0u && shiftm == 0u && tcol[0] >= 0 && tcol[1] >= 0 &&
                        tcol[2] >= 0;
    if (__ballot(!tab_ok) == 0ull) {
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
            const int v = L::ex[i] + 1;
            const int src = ((L::DIM == 3 ? (1 - L::ez[i]) * rs.TY : 0) + 1 - L::ey[i]) * rs.nwd + tcol[v];
            const unsigned lo = __shfl((unsigned)(rs.wm & 0xffffffffull), src, 64);
            const unsigned hi = __shfl((unsigned)(rs.wm >> 32), src, 64);
            const int pb = __shfl(rs.wpb, src, 64);
            const unsigned long long m = ((unsigned long long)hi << 32) | lo;
            const unsigned long long bit = tbit[v];
            kk[i] = (m & bit) ? pb + __popcll(m & (bit - 1ull)) : -1;
            if (kk[i] == -1) solidnb |= 1u << i;
        }
        return;
    }
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const int v = L::ex[i] + 1;
        const bool in_tab = tcol[v] >= 0;
        const int src = in_tab ? ((L::DIM == 3 ? (1 - L::ez[i]) * rs.TY : 0) + 1 - L::ey[i]) * rs.nwd + tcol[v] : 0;
        const unsigned lo = __shfl((unsigned)(rs.wm & 0xffffffffull), src, 64);
        const unsigned hi = __shfl((unsigned)(rs.wm >> 32), src, 64);
        const int pb = __shfl(rs.wpb, src, 64);
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

}  // namespace lbm
