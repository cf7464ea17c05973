// Host-only check of the library's device-layout construction (no GPU): reads
// hierarchy files with the library's own parser, builds the layouts the
// upload would build (optionally for the block-diagonal union of several
// files, as a batch upload does) and checks their invariants.  Built by the
// CPU test suite with AddressSanitizer.
//
// usage: layout_check [--batch] file...   prints "ok <summary>" or fails
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hier_host.hpp"

using namespace mvamg;

static int fails = 0;
#define CHECK(c, msg)                                                 \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed: %s (%s)\n", msg, #c);       \
      if (++fails > 20) return 1;                                     \
    }                                                                 \
  } while (0)

static int check_level(const HostLevel& L, const LevelLayout& Y, const std::vector<int>* rowprob) {
  const int n = L.n;
  CHECK((int)Y.perm.size() == n && (int)Y.iperm.size() == n, "permutation size");
  for (int p = 0; p < n; ++p) CHECK(Y.iperm[Y.perm[p]] == p, "perm/iperm inverse");
  const int ng = (int)Y.gstart.size() - 1, ns = (int)Y.sgrp.size() - 1;
  CHECK(Y.gstart[0] == 0 && Y.gstart[ng] == n, "groups cover the rows");
  CHECK(Y.sgrp[0] == 0 && Y.sgrp[ns] == ng, "stages cover the groups");
  // every row's stored entries (off-group + diagonal block) reproduce its CSR row sum and |.| sum
  std::vector<int> grp(n);
  for (int g = 0; g < ng; ++g)
    for (int p = Y.gstart[g]; p < Y.gstart[g + 1]; ++p) grp[p] = g;
  std::vector<double> s1(n, 0.0), s2(n, 0.0);
  for (int g = 0; g < ng; ++g) {
    const int k = Y.gstart[g + 1] - Y.gstart[g];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        const double v = Y.dblk[Y.dboff[g] + a * k + b];
        s1[Y.gstart[g] + a] += v;
        s2[Y.gstart[g] + a] += std::fabs(v);
      }
  }
  if (Y.sell) {
    CHECK((int)Y.sslab.size() == ns + 1, "stage slab ranges");
    for (int c = 0; c < ns; ++c) {
      int next = Y.gstart[Y.sgrp[c]];
      for (int q = Y.sslab[c]; q < Y.sslab[c + 1]; ++q) {
        const Slab& sl = Y.slabs[q];
        CHECK(sl.row0 == next && sl.nrows >= 1 && sl.nrows <= 64, "slabs tile the stage in order");
        next += sl.nrows;
        if (rowprob)
          for (int i = 1; i < sl.nrows; ++i)
            CHECK((*rowprob)[Y.perm[sl.row0 + i]] == (*rowprob)[Y.perm[sl.row0]], "slab inside one problem");
        for (int i = 0; i < sl.nrows; ++i) {
          const int p = sl.row0 + i, r = Y.perm[p];
          CHECK(sl.width >= L.rp[r + 1] - L.rp[r] - 1, "slab width covers the row");
          for (int j = 0; j < sl.width; ++j) {
            const int64_t at = (int64_t)sl.off + (int64_t)j * 64 + i;
            CHECK(at >= 0 && at < (int64_t)Y.col.size(), "slab entry in range");
            CHECK(Y.col[at] >= 0 && Y.col[at] < n, "slab column in range");
            s1[p] += Y.val[at];
            s2[p] += std::fabs(Y.val[at]);
          }
        }
      }
      CHECK(next == Y.gstart[Y.sgrp[c + 1]], "slabs end with the stage");
    }
    // 16-bit column deltas reproduce every stored column; padding points at a row
    CHECK(Y.scb.size() == Y.slabs.size() && Y.pk.size() == Y.slabs.size(), "16-bit column arrays");
    int64_t packed = 0;
    for (size_t q = 0; q < Y.slabs.size(); ++q) {
      CHECK(Y.pk[q] == packed && Y.pk[q] % 512 == 0, "packed slab offsets");
      packed += (int64_t)(Y.slabs[q].width + 7) / 8 * 512;
    }
    CHECK((int64_t)Y.col16.size() == packed && (!Y.vcoded || (int64_t)Y.vcode.size() == packed), "packed sizes");
    int64_t real16 = 0;
    for (size_t q = 0; q < Y.slabs.size(); ++q) {
      if (Y.scb[q] < 0) continue;
      const Slab& sl = Y.slabs[q];
      const int cb = Y.scb[q];
      CHECK(cb >= 0 && (size_t)cb + (size_t)((sl.width + 7) / 8 * 8) <= Y.cbase.size(), "bases padded to 8");
      for (int i = 0; i < sl.nrows; ++i) {
        const int r = Y.perm[sl.row0 + i], len = L.rp[r + 1] - L.rp[r] - 1;
        for (int j = 0; j < sl.width; ++j) {
          const int64_t at = (int64_t)sl.off + (int64_t)j * 64 + i;
          const int64_t c16 = (int64_t)Y.cbase[cb + j] + Y.col16[pk_index(Y, (int)q, j, i)];
          if (j < len) {
            CHECK(c16 == Y.col[at], "16-bit column equals the stored column");
            ++real16;
          } else {
            CHECK(c16 >= 0 && c16 < n && Y.val[at] == 0.0, "16-bit padding points at a row, value 0");
          }
        }
        // packed slots past the width (read by the eight-slot loads, products dropped) point at a row
        for (int j = sl.width; j < (sl.width + 7) / 8 * 8; ++j) {
          const int64_t c16 = (int64_t)Y.cbase[cb + j] + Y.col16[pk_index(Y, (int)q, j, i)];
          CHECK(c16 >= 0 && c16 < n, "packed padding slot points at a row");
        }
      }
    }
    CHECK(real16 == Y.nnz16, "16-bit entry count");
    // value dictionaries decode to the stored values bit for bit
    if (Y.vcoded) {
      CHECK(!Y.vtab.empty() && Y.vtab.size() <= 256, "entry codes");
      for (size_t q = 0; q < Y.slabs.size(); ++q) {
        const Slab& sl = Y.slabs[q];
        for (int j = 0; j < (sl.width + 7) / 8 * 8; ++j)
          for (int i = 0; i < 64; ++i) {
            const uint8_t c = Y.vcode[pk_index(Y, (int)q, j, i)];
            CHECK(c < Y.vtab.size(), "code inside the table");
            if (j < sl.width)
              CHECK(std::memcmp(&Y.vtab[c], &Y.val[(int64_t)sl.off + (int64_t)j * 64 + i], sizeof(double)) == 0,
                    "entry code decodes to the value");
          }
      }
    }
    if (Y.dcoded) {
      CHECK(Y.dcode.size() == Y.dblk.size() && (int)Y.dblk.size() == n && Y.dtab.size() <= 256, "diagonal codes");
      for (size_t i = 0; i < Y.dblk.size(); ++i)
        CHECK(Y.dcode[i] < Y.dtab.size() && std::memcmp(&Y.dtab[Y.dcode[i]], &Y.dblk[i], sizeof(double)) == 0,
              "diagonal code decodes to the value");
    }
  } else {
    CHECK((int)Y.rowptr.size() == n + 1 && Y.rowptr[n] == (int)Y.col.size(), "grouped CSR");
    // a row's entries in increasing column order; rsplit separates the entries
    // of earlier stages from those of later stages
    CHECK((int)Y.rsplit.size() == n, "row splits");
    std::vector<int> stage_of(n, 0);
    for (int c = 0; c < ns; ++c)
      for (int p = Y.gstart[Y.sgrp[c]]; p < Y.gstart[Y.sgrp[c + 1]]; ++p) stage_of[p] = c;
    for (int p = 0; p < n; ++p) {
      const int later = Y.gstart[Y.sgrp[stage_of[p] + 1]];
      CHECK(Y.rsplit[p] >= Y.rowptr[p] && Y.rsplit[p] <= Y.rowptr[p + 1], "split inside the row");
      for (int e = Y.rowptr[p]; e < Y.rowptr[p + 1]; ++e) {
        if (e > Y.rowptr[p]) CHECK(Y.col[e - 1] < Y.col[e], "row entries in increasing column order");
        CHECK((e < Y.rsplit[p]) == (Y.col[e] < later), "split separates earlier and later stages");
      }
    }
    // the kernels' index lists: entry e of row l of group g at gcol[e + gcsh[g] - l gcm[g]]
    const int ngr = (int)Y.gstart.size() - 1;
    CHECK((int)Y.gcsh.size() == ngr && (int)Y.gcm.size() == ngr, "group index records");
    int64_t saved = 0, stored = 0;
    for (int g = 0; g < ngr; ++g) {
      const int p0 = Y.gstart[g], k = Y.gstart[g + 1] - p0;
      for (int l = 0; l < k; ++l) {
        if (Y.gcm[g] > 0) CHECK(Y.rowptr[p0 + l + 1] - Y.rowptr[p0 + l] == Y.gcm[g], "shared row length");
        for (int e = Y.rowptr[p0 + l]; e < Y.rowptr[p0 + l + 1]; ++e) {
          const int64_t at = (int64_t)e + Y.gcsh[g] - (int64_t)l * Y.gcm[g];
          CHECK(at >= 0 && at < (int64_t)Y.gcol.size() && Y.gcol[at] == Y.col[e], "group index list");
        }
      }
      stored += Y.gcm[g] > 0 ? Y.gcm[g] : Y.rowptr[p0 + k] - Y.rowptr[p0];
      saved += Y.gcm[g] > 0 ? (int64_t)(k - 1) * Y.gcm[g] : 0;
    }
    int64_t sstored = 0;
    for (int c = 0; c < ns; ++c) sstored += Y.stage_gidx[c];
    CHECK(stored == (int64_t)Y.gcol.size() && sstored == stored && saved + stored == (int64_t)Y.col.size(),
          "group index list sizes");
    for (int p = 0; p < n; ++p)
      for (int e = Y.rowptr[p]; e < Y.rowptr[p + 1]; ++e) {
        const int q = Y.col[e];
        CHECK(q >= 0 && q < n && grp[q] != grp[p], "off-group entry");
        s1[p] += Y.val[e];
        s2[p] += std::fabs(Y.val[e]);
      }
  }
  for (int p = 0; p < n; ++p) {
    const int r = Y.perm[p];
    double t1 = 0.0, t2 = 0.0;
    for (int e = L.rp[r]; e < L.rp[r + 1]; ++e) {
      t1 += L.v[e];
      t2 += std::fabs(L.v[e]);
    }
    CHECK(std::fabs(s1[p] - t1) <= 1e-12 * (t2 + 1e-300) + 1e-300 && std::fabs(s2[p] - t2) <= 1e-12 * t2,
          "stored entries reproduce the row");
  }
  return 0;
}

int main(int argc, char** argv) {
  bool batch = false;
  std::vector<std::string> files;
  for (int i = 1; i < argc; ++i) {
    if (std::strcmp(argv[i], "--batch") == 0)
      batch = true;
    else
      files.push_back(argv[i]);
  }
  if (files.empty()) return 2;
  try {
    std::vector<HostHier> Hs;
    for (const std::string& f : files) Hs.push_back(read_hierarchy_file(f.c_str()));
    std::vector<HostHier> todo;
    std::vector<std::vector<int>> rowprob(1);
    if (batch) {
      std::vector<const HostHier*> ptr;
      for (const HostHier& H : Hs) ptr.push_back(&H);
      todo.push_back(union_hierarchy(ptr));
      for (size_t p = 0; p < Hs.size(); ++p) rowprob[0].insert(rowprob[0].end(), Hs[p].lv[0].n, (int)p);
      // the union is block diagonal: rows of problem p only couple rows of problem p
      const HostLevel& U0 = todo[0].lv[0];
      for (int i = 0; i < U0.n; ++i)
        for (int e = U0.rp[i]; e < U0.rp[i + 1]; ++e) CHECK(rowprob[0][U0.ci[e]] == rowprob[0][i], "union is block diagonal");
    } else {
      todo = Hs;
    }
    for (const HostHier& H : todo) {
      std::vector<LevelLayout> Y(H.nl - 1);
      for (int l = 0; l + 1 < H.nl; ++l) {
        build_level_layout(H.lv[l], Y[l], (batch && l == 0) ? &rowprob[0] : nullptr);
        if (check_level(H.lv[l], Y[l], (batch && l == 0) ? &rowprob[0] : nullptr)) return 1;
      }
      for (int l = 0; l + 1 < H.nl; ++l) {
        TransferLayout T;
        build_transfer_layout(H.lv[l], Y[l], (l + 2 < H.nl) ? &Y[l + 1] : nullptr, T);
        int64_t cover = 0;
        for (int a = 0; a < T.nagg; ++a) {
          CHECK(T.kk[a] >= 1 && T.kk[a] <= kKmax, "block width");
          CHECK(T.cst[a] >= 0 && T.cst[a] + T.kk[a] <= H.lv[l + 1].n, "coarse rows in range");
          cover += T.kk[a];
        }
        CHECK(cover == H.lv[l + 1].n, "aggregates cover the coarse level");
      }
      long long gsh = 0, gall = 0;  // groups of grouped levels, and those with a shared column list
      for (int l = 0; l + 1 < H.nl; ++l)
        if (!Y[l].sell)
          for (int m : Y[l].gcm) {
            gall += 1;
            gsh += m > 0;
          }
      std::printf("ok levels=%d n0=%d sell0=%d nnz16_0=%lld nnz0=%lld gshared=%lld/%lld coded0=%d%d\n", H.nl,
                  H.lv[0].n, H.nl > 1 ? (int)Y[0].sell : -1, H.nl > 1 ? (long long)Y[0].nnz16 : 0LL,
                  (long long)H.lv[0].rp[H.lv[0].n] - H.lv[0].n, gsh, gall, H.nl > 1 ? (int)Y[0].vcoded : 0,
                  H.nl > 1 ? (int)Y[0].dcoded : 0);
    }
  } catch (const std::exception& e) {
    std::fprintf(stderr, "error: %s\n", e.what());
    return 3;
  }
  return fails ? 1 : 0;
}
