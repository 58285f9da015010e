// Index arithmetic of the field-solver kernels: partial-sum slots, the row -> slot maps of the
// block flushes, the layout of each system's small FP64 block, and the map from a block of the
// register-resident step kernels to its (system, chunk).  The kernels call these functions, and
// a host-side bounds check (tests/index_bounds.cpp) compiles this same header with a plain C++
// compiler, so it holds no device builtins.
#pragma once

#include <stddef.h>

#ifdef __HIPCC__
#define HYDOT_HD __host__ __device__
#else
#define HYDOT_HD
#endif

namespace hydot {

constexpr int kMaxK = 32;                  // recycle dimension
constexpr int kMaxMK = 128;                // Arnoldi steps per cycle (also Lanczos steps)
constexpr int kMaxDots = 3 * kMaxK + kMaxMK + 2;

// ----------------------------------------------------------------- partial-sum slots
// Per (system, chunk) the kernels write ndots FP64 partial sums: the deflation products
// C'_i^H w in slots 3i + c (c = 0; the generic kernels also use c = 1, 2 for C^T w, U^T w and
// (rho U)^T w), the basis products V_l^H w in 3k + l, and |w|^2 in 3k + mkmax + 1.
HYDOT_HD inline int slot_defl(int i, int c) { return 3 * i + c; }
HYDOT_HD inline int slot_v(int k, int l) { return 3 * k + l; }
HYDOT_HD inline int slot_norm(int k, int mkmax) { return 3 * k + mkmax + 1; }
HYDOT_HD inline int ndots_for(int k, int mkmax) { return 3 * k + mkmax + 2; }

// first partial sum of (system, chunk): partials are [system][chunk][ndots]
HYDOT_HD inline size_t part_base(int sys, int nchunks, int chunk, int ndots) {
  return ((size_t)sys * nchunks + chunk) * ndots;
}

// Row -> slot of the single-round product tile (at most 16 basis vectors): rows [0, nv) the
// basis products, rows [nv, nv + k) the deflation products, row nv + k the norm.
HYDOT_HD inline int flush_all_slot(int row, int nv, int k, int mkmax) {
  if (row < nv) return slot_v(k, row);
  if (row < nv + k) return slot_defl(row - nv, 0);
  return slot_norm(k, mkmax);
}
// Row -> slot of a tile of rows slot0 + 3 row (the deflation rows of the two-round form), with
// the norm in row norm_row (-1: none).
HYDOT_HD inline int flush_rows_slot(int row, int slot0, int norm_row, int k, int mkmax) {
  return row == norm_row ? slot_norm(k, mkmax) : slot0 + 3 * row;
}
// Row -> slot of the basis-product tile of the two-round form.
HYDOT_HD inline int flush_v_slot(int row, int k) { return slot_v(k, row); }

// ----------------------------------------------------------------- small per-system block
// Offsets (in complex-double units) inside one system's small block.
struct Small {
  int coefA, coefB, H, cs, sn, gam, Fp, vs, Lc, y0, cA32, total;
};

HYDOT_HD inline Small make_small(int k, int mkmax, int nl) {
  Small s;
  int o = 0;
  s.coefA = o; o += k + mkmax + 2;
  s.coefB = o; o += k + mkmax + 2;
  s.H = o; o += (mkmax + 1) * mkmax;
  s.cs = o; o += mkmax;
  s.sn = o; o += mkmax;
  s.gam = o; o += mkmax + 1;
  s.Fp = o; o += k * mkmax;
  s.vs = o; o += mkmax + 2;      // basis scales: v_l = vs[l] * (stored V_l)
  s.Lc = o; o += k * k;          // y0 follows Lc directly (one host copy fills both)
  s.y0 = o; o += (nl > 0 ? nl : 1);
  s.cA32 = o; o += (k + mkmax + 3) / 2;   // FP32 copy of the step coefficients coefA (complex float)
  s.total = (o + 15) & ~15;
  return s;
}

// Element offsets of the small-block arrays the reduce kernel indexes.
HYDOT_HD inline int small_H(const Small& s, int mkmax, int i, int j) { return s.H + i + (mkmax + 1) * j; }
HYDOT_HD inline int small_Fp(const Small& s, int k, int i, int j) { return s.Fp + i + k * j; }

// ----------------------------------------------------------------- block -> (system, chunk)
constexpr int kChunkVoxels = 2048;   // voxels per (system, chunk) tile of the step kernels

// Default block order of a grid: the chunk-per-XCD order (4) where a z-plane holds a multiple of
// 8 chunks, so that chunk c and its z-neighbour chunks c +- nx ny / 2048 share XCD c % 8;
// elsewhere the z-slab order (3).
HYDOT_HD inline int default_step_order(int nx, int ny) {
  return ((long long)nx * ny) % (8 * kChunkVoxels) == 0 ? 4 : 3;
}

struct TileIdx {
  int sys, chunk;
};
// Block b of nblk = nb * nchunks blocks, in groups of grp systems (nb a multiple of grp).
// flags bit 0: XCD-contiguous order; bit 1: z-slab order; bit 2: chunk-per-XCD order with the
// systems of a group adjacent (takes precedence over bits 0 and 1).
// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// XCD-contiguous: each XCD gets a contiguous range of the logical order (whole systems), at the
// price of reading a right-hand side's C and U on every XCD.
// z-slab: the logical chunk position q lands on XCD (q * grp + system) % 8, a class of q mod Q
// (Q = 8 / gcd(grp, 8)) when grp * nchunks is a multiple of 8.  Class x is given the x-th
// contiguous range of chunks, i.e. a slab of z-planes: the stencil's z-neighbour chunks are then
// read on the same XCD, by blocks a few dispatch slots apart, and hit its L2; the chunks of one
// right-hand side still stay on one XCD.
// Chunk-per-XCD order (bit 2, when the chunk count is a multiple of 8): chunk c always runs on
// XCD c % 8, so the stencil's z-neighbour chunks c +- 8 (a z-plane holds a multiple of 8 chunks
// on the large grids) are read on the same XCD; within an XCD the grp systems of one group (the
// wavelengths of one right-hand side, which share C and U) take one chunk in consecutive
// blocks, so that chunk of C and U is fetched once into that XCD's L2 and reused grp times.
HYDOT_HD inline TileIdx tile_map(int b, int nblk, int nchunks, int grp, int flags) {
  if ((flags & 4) && (nchunks & 7) == 0) {
    const int x = b & 7, i = b >> 3, nc8 = nchunks >> 3;
    const int s = i % grp, t = i / grp;
    return TileIdx{(t / nc8) * grp + s, (t % nc8) * 8 + x};
  }
  if ((flags & 1) && (nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int per = grp * nchunks;
  const int g = b / per, rem = b - g * per;
  int ch = rem / grp;
  if (flags & 2) {
    const int q8 = grp & 7;
    const int Q = q8 == 0 ? 1 : (q8 & 1) ? 8 : (q8 & 3) ? 4 : 2;
    if (Q > 1 && nchunks % Q == 0 && (per & 7) == 0) ch = (ch % Q) * (nchunks / Q) + ch / Q;
  }
  return TileIdx{g * grp + rem % grp, ch};
}

}  // namespace hydot
