// lbm_device.hpp -- lattices, the row-compressed fluid layout and site
// arithmetic shared by the gfx950 kernels.
//
// Velocity sets: D2Q9 in the order of the paper's appendix (velocity sets);
// D3Q19 as the rest vector, nine vectors and their negatives (e_{i+9} = -e_i).
// The populations exported through the C ABI use these orders.
//
// Layout.  Populations are stored for fluid nodes only, in node order, one
// contiguous array per direction ("compact index" k).  A fluid node's
// neighbours are found from per-row bit masks: the box is cut into x-rows
// (row = y + ny*z) and each row into 64-node words; for every word the
// library keeps the 64-bit fluid mask and the compact index of the first fluid
// node of the word (RowWord, 16 B per 64 nodes).  The compact index of the
// fluid node at x in row r is pb + popcount(mask & ((1 << (x & 63)) - 1)) of
// word (r, x >> 6).  One wavefront processes up to 64 consecutive fluid nodes
// (a "task") of one row, or of a few consecutive rows of one plane when their
// fluid nodes fit together, so no lane is spent on a solid node and every
// load and store of a wavefront touches one contiguous range per direction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    static constexpr int ex[9] = {0, -1, -1, -1, 0, 1, 1, 1, 0};
    static constexpr int ey[9] = {0, 1, 0, -1, -1, -1, 0, 1, 1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9,
                                    1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    static constexpr int ex[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
    static constexpr int ey[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
    static constexpr int ez[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
    static constexpr int opp[19] = {0, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                                    1, 2, 3, 4, 5, 6, 7, 8, 9};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

constexpr int BLK = 256;

// bit mask of the directions whose component along axis a (0 x, 1 y, 2 z) is s
template <class L>
__host__ __device__ constexpr uint32_t dir_mask(int a, int s) {
    uint32_t m = 0u;
    for (int i = 0; i < L::Q; i++)
        if ((a == 0 ? L::ex[i] : a == 1 ? L::ey[i] : L::ez[i]) == s) m |= 1u << i;
    return m;
}

// Solute velocity sets.  The solute runs on the fluid's own set, or on the
// paper's reduced D2Q5 / D3Q7 (appendix, velocity sets): the rest vector and
// the unit vectors along the axes, a subset of D2Q9 / D3Q19.  A set is a bit
// mask over the fluid directions.  Solute populations are stored for the
// set's directions only: slot s holds the s-th direction of the mask (for
// D2Q5 the paper's order, for D3Q7 rest, +x, +y, +z, -x, -y, -z).
template <class L>
__host__ __device__ constexpr uint32_t axis_mask() {
    uint32_t m = 0u;
    for (int i = 0; i < L::Q; i++)
        if (L::ex[i] * L::ex[i] + L::ey[i] * L::ey[i] + L::ez[i] * L::ez[i] <= 1) m |= 1u << i;
    return m;
}

template <class L, bool RED>
__host__ __device__ constexpr uint32_t sol_mask() {
    return RED ? axis_mask<L>() : (1u << L::Q) - 1u;
}

// storage slot of fluid direction i in the solute set m
__host__ __device__ constexpr int sol_slot(uint32_t m, int i) {
    return __builtin_popcount(m & ((1u << i) - 1u));
}

// Population arrays are blocked by 64 fluid nodes: [k / 64][slot][k % 64]
// for nq slots per node (Q for the fluid, QS for the solute and the adjoint).
// A wavefront's 64 consecutive nodes find every direction of theirs in one
// contiguous stretch of nq * 256 B (FP32), instead of nq streams a full
// array apart.  The arrays hold nq * S elements (S a multiple of 64).
__host__ __device__ __forceinline__ long pidx(int slot, long k, int nq) {
    return ((k >> 6) * nq + slot) * 64 + (k & 63);
}

// Wait for every outstanding vector memory operation of the wavefront,
// global-to-LDS loads included.  The compiler does not order an LDS read after
// the global-to-LDS load that fills its location (it may issue the read right
// behind it), so a kernel that stages data that way calls this before its
// first read of the staged data, at a point where it waits for its own loads
// anyway.  The asm is a wait instruction, with a memory clobber so that no
// LDS read is moved above it.
__device__ __forceinline__ void lds_dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Element index of slot 0 of node k (slot s is 64 s further): pidx() with one
// 32 x 32 -> 64-bit multiply, for a compact index k >= 0.  Kernels form a
// node's own base once and reuse it for every slot.
__device__ __forceinline__ long blk0(int k, int nq) {
    return (long)((unsigned long long)((unsigned)k >> 6) * (unsigned)(nq * 64)) + (k & 63);
}

// Node flags of the geometry pass (dense, uint32 per node; not read per step)
//   bits 0..Q-1 : fluid view, upstream site x - e_i is solid or outside a
//                 non-periodic face
//   bit 30      : node has at least one reactive link
//   bit 31      : node is fluid
constexpr uint32_t F_LINK = 1u << 30;
constexpr uint32_t F_FLUID = 1u << 31;

struct RowWord {
    unsigned long long mask;   // bit b: node x = 64*w + b of the row is fluid
    int32_t pb;                // compact index of the first fluid node of the word
    int32_t pad;
};

struct Task {
    int32_t row;               // first row of the task (of its domain), y + ny*z
    int32_t k0;                // compact index of the task's first node
    int32_t cnt;               // nodes in the task (1..64) | rows spanned << 8
    int32_t dom;               // domain of the batch
    int32_t wlo, nwd;          // window of row words the task's table holds
    int32_t y0, z;             // the first row's y and z (row = y0 + ny*z)
};

struct Box {
    int nx, ny, nz;
    int per[3];        // fluid periodicity
    int shift;         // site (x + nx, y) is site (x, y + shift)
    int inlet_axis;    // solute: non-periodic axis with inlet/outlet, or -1
};

// One domain of a batch, as the kernels see it (a single lattice is a batch of
// one).  Dense node arrays of all domains are concatenated in domain order, as
// are their row words and their compact fluid arrays.
struct DomDev {
    Box box;
    int W;                     // 64-node words per row
    int mech, scheme;
    long node_off;             // first dense node of the domain
    long word_off;             // first row word of the domain
    long row_off;              // first global row of the domain
    double omega_f, omega_g, force_fac;
    // TRT (trt = 1): fluid odd parts relax with omega_fm, their force share
    // scaled by force_fac_m; solute even parts relax with omega_gs (odd ones
    // with omega_g).  BGK: omega_fm = omega_f, omega_gs = omega_g
    int trt;
    uint32_t smask;            // solute velocity set (bit i: fluid direction i)
    int fopen;                 // open channel along the inlet axis (plug inflow u_in,
    double u_in, rho_out;      // outlet density rho_out)
    double omega_fm, force_fac_m, omega_gs;
    double F[3];
    double ws[19];             // solute weights by fluid direction (rest fraction;
                               // 0 outside the solute set)
    double wsc;                // ws[i] = w[i] * wsc for every moving direction of the set
    double inv_cs2s, cs2s, gamma;
    double rho0, c_ref;        // deviation references (0 in FP64 storage)
    double ceq_dev;            // C_eq - C_ref
    double c_in;
    double vma;                // V_m a_m
    double v_m;                // molar volume (phase change)
    double kr0;                // uniform rate constant
};

// solute weight of direction i: the rest weight is stored, the moving ones are
// the lattice weights times one scale (keeps the step kernel's constants few)
template <class L>
__device__ __forceinline__ double sol_w(const DomDev &D, int i) {
    return i == 0 ? D.ws[0] : L::w[i] * D.wsc;
}

// domain of dense node n (off: node_off of every domain, then the total)
__device__ inline int find_dom(const long *off, int ndom, long n) {
    int lo = 0, hi = ndom;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= n) lo = mid;
        else hi = mid;
    }
    return lo;
}

__host__ __device__ inline int fdiv(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Wrap (x, y, z) into the box under the fluid's periodicity.  Returns false,
// with *face = 2*axis + (1 on the high side), when the site is outside a
// non-periodic face.
__host__ __device__ inline bool wrap_site(const Box &b, int &x, int &y, int &z, int *face) {
    *face = -1;
    if (x < 0 || x >= b.nx) {
        if (!b.per[0]) { *face = x < 0 ? 0 : 1; return false; }
        const int k = fdiv(x, b.nx);
        x -= k * b.nx;
        y += k * b.shift;
    }
    if (y < 0 || y >= b.ny) {
        if (!b.per[1]) { *face = y < 0 ? 2 : 3; return false; }
        y -= fdiv(y, b.ny) * b.ny;
    }
    if (z < 0 || z >= b.nz) {
        if (!b.per[2]) { *face = z < 0 ? 4 : 5; return false; }
        z -= fdiv(z, b.nz) * b.nz;
    }
    return true;
}

// Dense node index of the site reached from (x,y,z) by (dx,dy,dz), or -1 when
// it leaves the box through a face that is not periodic in this view (the
// solute sees the inlet axis as non-periodic).
__host__ __device__ inline long site(const Box &b, int x, int y, int z, int dx, int dy, int dz,
                                     bool solute, int *face) {
    int c[3] = {x + dx, y + dy, z + dz};
    if (solute && b.inlet_axis >= 0) {
        const int a = b.inlet_axis;
        const int n = a == 0 ? b.nx : (a == 1 ? b.ny : b.nz);
        if (c[a] < 0 || c[a] >= n) { *face = 2 * a + (c[a] >= n ? 1 : 0); return -1; }
    }
    if (!wrap_site(b, c[0], c[1], c[2], face)) return -1;
    return (long)c[0] + (long)b.nx * ((long)c[1] + (long)b.ny * (long)c[2]);
}

__host__ __device__ inline void coords(const Box &b, long n, int *x, int *y, int *z) {
    const long nxy = (long)b.nx * b.ny;
    if (n >= 0 && n <= 0xffffffffL && nxy <= 0xffffffffL) {
        // 32-bit quotients (a 64-bit division is a long software sequence)
        const unsigned un = (unsigned)n, uxy = (unsigned)nxy, unx = (unsigned)b.nx;
        const unsigned zz = un / uxy, r = un - zz * uxy, yy = r / unx;
        *z = (int)zz;
        *y = (int)yy;
        *x = (int)(r - yy * unx);
        return;
    }
    *z = (int)(n / nxy);
    const long r = n - (long)(*z) * nxy;
    *y = (int)(r / b.nx);
    *x = (int)(r - (long)(*y) * b.nx);
}

// Workgroup id remapped so that consecutive tiles of work run on the same XCD
// (gfx950 dispatches workgroups round-robin over its 8 XCDs; each XCD has its
// own L2, and neighbouring tiles share the cache lines at their edges).
__device__ inline long xcd_tile(long hw, long nblocks) {
    const long nx = 8;
    const long xcd = hw % nx, local = hw / nx;
    const long base = nblocks / nx, rem = nblocks % nx;
    const long start = xcd * base + (xcd < rem ? xcd : rem);
    return start + local;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over a workgroup of BLK threads; result valid in thread 0.  Every thread
// of the workgroup must call it.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[BLK / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BLK / 64; k++) s += part[k];
    __syncthreads();
    return s;
}

}  // namespace lbm
