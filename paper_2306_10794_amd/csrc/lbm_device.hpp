// lbm_device.hpp -- lattices, node flags and site arithmetic for the gfx950 kernels.
//
// Velocity sets: D2Q9 in the order of the paper's appendix (velocity sets);
// D3Q19 as the rest vector, nine vectors and their negatives (e_{i+9} = -e_i).
// The populations exported through the C ABI use these orders.
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

// Node flags (uint32 per node)
//   bits 0..Q-1 : fluid view, upstream site x - e_i is solid or outside a
//                 non-periodic face (halfway bounce-back for the fluid)
//   bit 29      : node lies on a face of the box (site arithmetic must wrap)
//   bit 30      : node has at least one reactive link
//   bit 31      : node is fluid
constexpr uint32_t F_FACE = 1u << 29;
constexpr uint32_t F_LINK = 1u << 30;
constexpr uint32_t F_FLUID = 1u << 31;
constexpr uint32_t F_DIRS = (1u << 19) - 1u;

// classes of an incoming solute population at a fluid node
constexpr int C_KNOWN = 0;   // pulled from a fluid site
constexpr int C_RBC = 1;     // upstream site is solid inside the box: reactive link
constexpr int C_WALL = 2;    // outside a non-periodic face: plain bounce-back
constexpr int C_INLET = 3;   // outside the low face of the inlet axis
constexpr int C_OUTLET = 4;  // outside the high face of the inlet axis

struct Box {
    int nx, ny, nz;
    int per[3];        // fluid periodicity
    int shift;         // (x + nx, y) is (x, y + shift)
    int inlet_axis;    // solute: non-periodic axis with inlet/outlet, or -1
};

__host__ __device__ inline int fdiv(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Site reached from (x,y,z) by (dx,dy,dz).  Returns the node index, or -1
// with *face = 2*axis + (1 on the high side) when the move leaves the box
// through a face that is not periodic in this view (solute: the inlet axis is
// never periodic).
__host__ __device__ inline long site(const Box &b, int x, int y, int z, int dx, int dy,
                                     int dz, bool solute, int *face) {
    int c0 = x + dx, c1 = y + dy, c2 = z + dz;
    *face = -1;
    if (c0 < 0 || c0 >= b.nx) {
        if (!b.per[0] || (solute && b.inlet_axis == 0)) { *face = c0 < 0 ? 0 : 1; return -1; }
        int k = fdiv(c0, b.nx);
        c0 -= k * b.nx;
        c1 += k * b.shift;
    }
    if (c1 < 0 || c1 >= b.ny) {
        if (!b.per[1] || (solute && b.inlet_axis == 1)) { *face = c1 < 0 ? 2 : 3; return -1; }
        c1 -= fdiv(c1, b.ny) * b.ny;
    }
    if (c2 < 0 || c2 >= b.nz) {
        if (!b.per[2] || (solute && b.inlet_axis == 2)) { *face = c2 < 0 ? 4 : 5; return -1; }
        c2 -= fdiv(c2, b.nz) * b.nz;
    }
    return (long)c0 + (long)b.nx * ((long)c1 + (long)b.ny * (long)c2);
}

__host__ __device__ inline void coords(const Box &b, long n, int *x, int *y, int *z) {
    long nxy = (long)b.nx * b.ny;
    *z = (int)(n / nxy);
    long r = n - (long)(*z) * nxy;
    *y = (int)(r / b.nx);
    *x = (int)(r - (long)(*y) * b.nx);
}

// Workgroup id remapped so that consecutive tiles of the node range run on the
// same XCD (gfx950 dispatches workgroups round-robin over its 8 XCDs; each XCD
// has its own L2, and neighbouring tiles share the cache lines at their edges).
__device__ inline long xcd_tile(long hw, long nblocks) {
    const long nx = 8;
    long xcd = hw % nx, local = hw / nx;
    long base = nblocks / nx, rem = nblocks % nx;
    long start = xcd * base + (xcd < rem ? xcd : rem);
    return start + local;
}

}  // namespace lbm
