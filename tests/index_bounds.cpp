// Host bounds check of the field solver's index arithmetic (paper_1410_0986_amd/csrc/krylov_index.h,
// the header the kernels use): partial-sum slots and the row -> slot maps of every flush, the
// per-system small block and every element the reduce kernel and the solver readback index in
// it, and the block -> (system, chunk) map of the register-resident step kernels, over every
// deflation dimension, cycle length, Lanczos length, basis count and block order the library
// accepts.  Prints "ok <checks>" and exits 0, or prints the first violation and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "krylov_index.h"

using namespace hydot;

static long long g_checks = 0;

#define REQUIRE(cond, ...)                                  \
  do {                                                      \
    ++g_checks;                                             \
    if (!(cond)) {                                          \
      std::printf("violation: %s: ", #cond);                \
      std::printf(__VA_ARGS__);                             \
      std::printf("\n");                                    \
      std::exit(1);                                         \
    }                                                       \
  } while (0)

// the register-resident kernels' limits (krylov_tiled.h): deflation rows, basis rows, tile rows
constexpr int kTK = 10, kTNV = 32, kTRows = 32;

static void check_slots(int k, int mkmax) {
  const int nd = ndots_for(k, mkmax);
  REQUIRE(nd <= kMaxDots, "k=%d mkmax=%d ndots=%d", k, mkmax, nd);
  std::vector<int> owner(nd, -1);
  // deflation slots 3i + c (c < 3: C'^H w, or C^T w, U^T w, (rho U)^T w in the generic kernels)
  for (int i = 0; i < k; ++i)
    for (int c = 0; c < 3; ++c) {
      const int s = slot_defl(i, c);
      REQUIRE(s >= 0 && s < nd && owner[s] == -1, "k=%d mkmax=%d defl %d %d", k, mkmax, i, c);
      owner[s] = 0;
    }
  // basis slots for every basis vector a step can hold (l <= mkmax: V_0..V_{mkmax})
  for (int l = 0; l <= mkmax; ++l) {
    const int s = slot_v(k, l);
    REQUIRE(s >= 0 && s < nd && owner[s] == -1, "k=%d mkmax=%d basis %d", k, mkmax, l);
    owner[s] = 1;
  }
  const int sn = slot_norm(k, mkmax);
  REQUIRE(sn >= 0 && sn < nd && owner[sn] == -1, "k=%d mkmax=%d norm", k, mkmax);
  // single-round tiles (at most 16 basis vectors, k <= kTK): rows nv + k + 1 in one tile
  if (k <= kTK) {
    for (int nv = 1; nv <= 16 && nv <= mkmax; ++nv) {
      const int nrows = nv + k + 1;
      REQUIRE(nrows <= kTRows, "k=%d nv=%d rows=%d", k, nv, nrows);
      std::vector<int> seen(nd, 0);
      for (int row = 0; row < nrows; ++row) {
        const int s = flush_all_slot(row, nv, k, mkmax);
        REQUIRE(s >= 0 && s < nd && !seen[s], "k=%d mkmax=%d nv=%d row=%d slot=%d", k, mkmax, nv, row, s);
        seen[s] = 1;
        const int expect = row < nv ? slot_v(k, row) : row < nv + k ? slot_defl(row - nv, 0) : sn;
        REQUIRE(s == expect, "k=%d nv=%d row=%d", k, nv, row);
      }
    }
    // two-round tiles (17..32 basis vectors): basis rows, then k deflation rows + the norm
    for (int nv = 17; nv <= kTNV && nv <= mkmax; ++nv) {
      REQUIRE(nv <= kTRows && k + 1 <= kTRows, "k=%d nv=%d", k, nv);
      std::vector<int> seen(nd, 0);
      for (int row = 0; row < nv; ++row) {
        const int s = flush_v_slot(row, k);
        REQUIRE(s >= 0 && s < nd && !seen[s], "k=%d nv=%d basis row %d", k, nv, row);
        seen[s] = 1;
      }
      for (int row = 0; row <= k; ++row) {
        const int s = flush_rows_slot(row, 0, k, k, mkmax);
        REQUIRE(s >= 0 && s < nd && !seen[s], "k=%d nv=%d defl row %d", k, nv, row);
        seen[s] = 1;
      }
    }
  }
  // reduce phases: the basis slots of step j are [slot_v(k, 0), slot_v(k, j + 1))
  for (int j = 0; j < mkmax; ++j) {
    const int lo = slot_v(k, 0), hi = slot_v(k, j + 1);
    REQUIRE(lo >= 0 && hi <= nd && lo <= hi && hi <= sn, "k=%d mkmax=%d j=%d", k, mkmax, j);
  }
}

static void check_lanczos_slots(int mkmax, int nl) {
  // Lanczos (k = 0): step j writes slots [0, j + 2) with slot j + 1 redirected to the norm slot
  const int nd = ndots_for(0, mkmax);
  for (int j = 0; j < nl; ++j) {
    for (int s = 0; s < j + 2; ++s) {
      const int o = s == j + 1 ? slot_norm(0, mkmax) : s;
      REQUIRE(o >= 0 && o < nd, "lanczos mkmax=%d j=%d s=%d", mkmax, j, s);
      REQUIRE(s == j + 1 || o == slot_v(0, s), "lanczos identity map");
    }
  }
}

static void check_small(int k, int mkmax, int nl) {
  const Small s = make_small(k, mkmax, nl);
  struct Region {
    int off, len;
    const char* name;
  } r[] = {{s.coefA, k + mkmax + 2, "coefA"}, {s.coefB, k + mkmax + 2, "coefB"}, {s.H, (mkmax + 1) * mkmax, "H"},
           {s.cs, mkmax, "cs"}, {s.sn, mkmax, "sn"}, {s.gam, mkmax + 1, "gam"}, {s.Fp, k * mkmax, "Fp"},
           {s.vs, mkmax + 2, "vs"}, {s.Lc, k * k, "Lc"}, {s.y0, nl > 0 ? nl : 1, "y0"},
           {s.cA32, (k + mkmax + 3) / 2, "cA32"}};
  const int nr = sizeof(r) / sizeof(r[0]);
  int end = 0;
  for (int i = 0; i < nr; ++i) {
    REQUIRE(r[i].off >= end && r[i].len >= 0, "k=%d mkmax=%d nl=%d region %s", k, mkmax, nl, r[i].name);
    end = r[i].off + r[i].len;
  }
  REQUIRE(end <= s.total && s.total % 16 == 0, "k=%d mkmax=%d nl=%d total", k, mkmax, nl);
  REQUIRE(s.y0 == s.Lc + k * k, "y0 must follow Lc (one host copy fills both)");
  auto in = [&](int idx, int ri) { return idx >= r[ri].off && idx < r[ri].off + r[ri].len; };
  // reduce kernel, every step j < mk (mk <= mkmax) and every cycle length ns <= mkmax
  for (int j = 0; j < mkmax; ++j) {
    for (int i = 0; i <= j + 1; ++i) REQUIRE(in(small_H(s, mkmax, i, j), 2), "H(%d,%d) k=%d mkmax=%d", i, j, k, mkmax);
    for (int i = 0; i < k; ++i) REQUIRE(in(small_Fp(s, k, i, j), 6), "Fp(%d,%d)", i, j);
    REQUIRE(in(s.coefA + k + j, 0), "coefA step coefficient j=%d", j);               // coef[k + l], l <= j
    REQUIRE(in(s.cs + j, 3) && 2 * j + 1 < 2 * mkmax, "cs j=%d", j);                  // double cs[2 j]
    REQUIRE(in(s.sn + j, 4), "sn j=%d", j);
    REQUIRE(in(s.gam + j + 1, 5), "gam j=%d", j);
    REQUIRE(in(s.vs + j + 1, 7), "vs j=%d", j);
    // FP32 copy of coefA: complex floats c32[i], i < k + j + 1, in (k + mkmax + 3) / 2 complex doubles
    REQUIRE(k + j + 1 <= 2 * ((k + mkmax + 3) / 2), "cA32 j=%d", j);
  }
  REQUIRE(in(s.coefB + k + mkmax + 1, 1), "coefB 1/eta slot");
  REQUIRE(in(s.gam + mkmax, 5), "gam cycle start, i <= mk");
  for (int q = 0; q < mkmax; ++q) REQUIRE(in(s.coefA + k + q, 0), "coefA cycle end q=%d", q);
  for (int i = 0; i < k; ++i)
    for (int q = 0; q < k; ++q) REQUIRE(in(s.Lc + i + k * q, 8), "Lc");
}

static void check_tiles(int nb, int nchunks, int grp, int flags) {
  const int nblk = nb * nchunks;
  std::vector<char> hit((size_t)nblk, 0);
  for (int b = 0; b < nblk; ++b) {
    const TileIdx t = tile_map(b, nblk, nchunks, grp, flags);
    REQUIRE(t.sys >= 0 && t.sys < nb && t.chunk >= 0 && t.chunk < nchunks,
            "nb=%d nchunks=%d grp=%d flags=%d b=%d -> (%d, %d)", nb, nchunks, grp, flags, b, t.sys, t.chunk);
    const size_t id = (size_t)t.sys * nchunks + t.chunk;
    REQUIRE(!hit[id], "nb=%d nchunks=%d grp=%d flags=%d: (%d, %d) twice", nb, nchunks, grp, flags, t.sys, t.chunk);
    hit[id] = 1;
  }
}

int main() {
  for (int k = 0; k <= kMaxK; ++k)
    for (int mkmax = 1; mkmax <= kMaxMK; ++mkmax) check_slots(k, mkmax);
  for (int mkmax = 1; mkmax <= kMaxMK; ++mkmax)
    for (int nl = 1; nl <= mkmax; ++nl) check_lanczos_slots(mkmax, nl);
  for (int k = 0; k <= kMaxK; ++k)
    for (int mkmax = 1; mkmax <= kMaxMK; ++mkmax)
      for (int nl : {0, 1, 7, 32, 40, mkmax}) check_small(k, mkmax, nl);
  // the step kernels' grids: chunks of 2048 voxels (the grids of every workload and ragged ones),
  // groups of 1 or of the L wavelengths of a right-hand side (the host takes grp > 1 only when
  // the batch is a multiple of it), every combination of the block-order bits
  const int chunk_counts[] = {1, 2, 3, 5, 7, 8, 12, 16, 24, 27, 64, 125, 216, 512};
  const int groups[] = {1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48, 64, 128};
  for (int nchunks : chunk_counts)
    for (int grp : groups)
      for (int mult : {1, 2, 3, 5, 8})
        for (int flags = 0; flags < 8; ++flags) {
          const int nb = grp * mult;
          if ((long long)nb * nchunks > 4000000) continue;
          check_tiles(nb, nchunks, grp, flags);
        }
  std::printf("ok %lld\n", g_checks);
  return 0;
}
