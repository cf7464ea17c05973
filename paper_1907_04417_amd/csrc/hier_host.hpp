// Host side of the library: hierarchy-file parser and the construction of the
// device layout (row permutation into smoother order, sliced-ELL or grouped
// CSR storage, per-group diagonal blocks, transfer descriptors).  Plain C++,
// no device code.  This parser is independent of the CPU oracle's reader.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

namespace mvamg {

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

// ------------------------------------------------------------ file parsing

struct HostLevel {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  std::vector<int> order, gptr, sptr;  // smoother order (non-coarsest levels)
  std::vector<int> aptr, arows, coff, uoff;  // transfer to the next level
  std::vector<double> U;
};

struct HostHier {
  int nl = 0, nvec = 0;
  std::vector<HostLevel> lv;
};

inline HostHier read_hierarchy_file(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) throw Error(-2, std::string("cannot open hierarchy file ") + path);
  std::vector<char> buf;
  {
    std::fseek(f, 0, SEEK_END);
    long sz = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    if (sz < 16) {
      std::fclose(f);
      throw Error(-2, "hierarchy file too short");
    }
    buf.resize((size_t)sz);
    size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got != buf.size()) throw Error(-2, "read error on hierarchy file");
  }
  if (std::memcmp(buf.data(), "MVAMGH01", 8) != 0) throw Error(-2, "bad magic in hierarchy file");
  uint32_t ver, nch;
  std::memcpy(&ver, buf.data() + 8, 4);
  std::memcpy(&nch, buf.data() + 12, 4);
  if (ver != 1) throw Error(-2, "unsupported hierarchy file version");
  struct Ch {
    uint32_t dtype;
    uint64_t count;
    size_t off;
  };
  std::map<std::string, Ch> ch;
  size_t off = 16;
  for (uint32_t c = 0; c < nch; ++c) {
    if (off + 64 > buf.size()) throw Error(-2, "truncated hierarchy file");
    char name[49] = {0};
    std::memcpy(name, buf.data() + off, 48);
    Ch e;
    std::memcpy(&e.dtype, buf.data() + off + 48, 4);
    std::memcpy(&e.count, buf.data() + off + 56, 8);
    off += 64;
    const size_t es = (e.dtype == 1) ? 4 : (e.dtype == 2 || e.dtype == 3) ? 8 : 0;
    if (!es) throw Error(-2, "unknown chunk type in hierarchy file");
    if (e.count > (buf.size() - off) / es) throw Error(-2, "truncated hierarchy file");
    e.off = off;
    off += es * e.count;
    off += (8 - (es * e.count) % 8) % 8;
    ch[name] = e;
  }
  auto get_i32 = [&](const std::string& nm, std::vector<int>& out) {
    auto it = ch.find(nm);
    if (it == ch.end() || it->second.dtype != 1) throw Error(-2, "missing chunk " + nm);
    out.resize(it->second.count);
    std::memcpy(out.data(), buf.data() + it->second.off, 4 * it->second.count);
  };
  auto get_f64 = [&](const std::string& nm, std::vector<double>& out) {
    auto it = ch.find(nm);
    if (it == ch.end() || it->second.dtype != 2) throw Error(-2, "missing chunk " + nm);
    out.resize(it->second.count);
    std::memcpy(out.data(), buf.data() + it->second.off, 8 * it->second.count);
  };
  auto it = ch.find("meta");
  if (it == ch.end() || it->second.dtype != 3 || it->second.count < 3) throw Error(-2, "missing meta chunk");
  int64_t meta[3];
  std::memcpy(meta, buf.data() + it->second.off, 24);
  HostHier H;
  H.nl = (int)meta[1];
  H.nvec = (int)meta[2];
  if (H.nl < 1 || H.nl > 32) throw Error(-2, "bad level count in hierarchy file");
  H.lv.resize(H.nl);
  for (int l = 0; l < H.nl; ++l) {
    HostLevel& L = H.lv[l];
    const std::string s = std::to_string(l);
    get_i32("A" + s + ".rowptr", L.rp);
    get_i32("A" + s + ".col", L.ci);
    get_f64("A" + s + ".val", L.v);
    L.n = (int)L.rp.size() - 1;
    if (L.n < 1 || L.rp[0] != 0 || (size_t)L.rp[L.n] != L.ci.size() || L.ci.size() != L.v.size())
      throw Error(-2, "inconsistent CSR arrays at level " + s);
    for (int i = 0; i < L.n; ++i) {
      if (L.rp[i + 1] < L.rp[i]) throw Error(-2, "rowptr not monotone at level " + s);
      for (int k = L.rp[i]; k < L.rp[i + 1]; ++k)
        if (L.ci[k] < 0 || L.ci[k] >= L.n) throw Error(-2, "column index out of range at level " + s);
    }
    if (l + 1 < H.nl) {
      get_i32("A" + s + ".order", L.order);
      get_i32("A" + s + ".gptr", L.gptr);
      get_i32("A" + s + ".sptr", L.sptr);
      get_i32("P" + s + ".aptr", L.aptr);
      get_i32("P" + s + ".arows", L.arows);
      get_i32("P" + s + ".coff", L.coff);
      get_i32("P" + s + ".uoff", L.uoff);
      get_f64("P" + s + ".U", L.U);
    }
  }
  // transfer consistency
  for (int l = 0; l + 1 < H.nl; ++l) {
    const HostLevel& L = H.lv[l];
    const int na = (int)L.aptr.size() - 1;
    const std::string s = std::to_string(l);
    if (na < 1 || (int)L.coff.size() != na + 1 || (int)L.uoff.size() != na + 1 || L.aptr[0] != 0 ||
        L.aptr[na] != L.n || (int)L.arows.size() != L.n || L.coff[0] != 0 ||
        L.coff[na] != H.lv[l + 1].n || L.uoff[0] != 0 || (size_t)L.uoff[na] != L.U.size())
      throw Error(-2, "inconsistent transfer arrays at level " + s);
    std::vector<char> seen(L.n, 0);
    for (int a = 0; a < na; ++a) {
      const int m = L.aptr[a + 1] - L.aptr[a], k = L.coff[a + 1] - L.coff[a];
      if (m < 1 || k < 1 || L.uoff[a + 1] - L.uoff[a] != m * k)
        throw Error(-2, "inconsistent aggregate at level " + s);
    }
    for (int q = 0; q < L.n; ++q) {
      const int i = L.arows[q];
      if (i < 0 || i >= L.n || seen[i]) throw Error(-2, "aggregates do not partition level " + s);
      seen[i] = 1;
    }
  }
  return H;
}

// Block-diagonal union of independent hierarchies with the same number of
// levels: level l of the union holds level l of every problem (rows of
// problem p after those of problems 0..p-1), stage c of its smoother order is
// stage c of every problem (groups and their order kept), and its aggregates
// are those of every problem.  A V-cycle of the union is the V-cycle of each
// problem, side by side.  The coarsest level's diagonal blocks are the
// problems' coarsest matrices.
inline HostHier union_hierarchy(const std::vector<const HostHier*>& Hs) {
  const int np = (int)Hs.size();
  if (np < 1) throw Error(-1, "empty batch");
  const int nl = Hs[0]->nl;
  for (const HostHier* H : Hs)
    if (H->nl != nl) throw Error(-1, "the problems of a batch must have the same number of levels");
  HostHier U;
  U.nl = nl;
  for (const HostHier* H : Hs) U.nvec = std::max(U.nvec, H->nvec);
  U.lv.resize(nl);
  std::vector<std::vector<int64_t>> off(nl, std::vector<int64_t>(np + 1, 0));
  for (int l = 0; l < nl; ++l)
    for (int p = 0; p < np; ++p) off[l][p + 1] = off[l][p] + Hs[p]->lv[l].n;
  for (int l = 0; l < nl; ++l) {
    if (off[l][np] >= ((int64_t)1 << 31)) throw Error(-1, "batch too large for 32-bit row indices");
    HostLevel& L = U.lv[l];
    L.n = (int)off[l][np];
    L.rp.assign(1, 0);
    for (int p = 0; p < np; ++p) {
      const HostLevel& S = Hs[p]->lv[l];
      const int o = (int)off[l][p];
      if ((int64_t)L.ci.size() + (int64_t)S.ci.size() >= ((int64_t)1 << 31))
        throw Error(-1, "batch too large for 32-bit entry offsets");
      for (int i = 0; i < S.n; ++i) {
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) {
          L.ci.push_back(S.ci[e] + o);
          L.v.push_back(S.v[e]);
        }
        L.rp.push_back((int)L.ci.size());
      }
    }
    if (l + 1 == nl) break;
    int ns = 0;
    for (int p = 0; p < np; ++p) ns = std::max(ns, (int)Hs[p]->lv[l].sptr.size() - 1);
    L.gptr.assign(1, 0);
    L.sptr.assign(1, 0);
    for (int c = 0; c < ns; ++c) {
      for (int p = 0; p < np; ++p) {
        const HostLevel& S = Hs[p]->lv[l];
        if (c + 1 >= (int)S.sptr.size()) continue;
        const int o = (int)off[l][p];
        for (int g = S.sptr[c]; g < S.sptr[c + 1]; ++g) {
          for (int q = S.gptr[g]; q < S.gptr[g + 1]; ++q) L.order.push_back(S.order[q] + o);
          L.gptr.push_back((int)L.order.size());
        }
      }
      L.sptr.push_back((int)L.gptr.size() - 1);
    }
    L.aptr.assign(1, 0);
    L.coff.assign(1, 0);
    L.uoff.assign(1, 0);
    int64_t ubase = 0;
    for (int p = 0; p < np; ++p) {
      const HostLevel& S = Hs[p]->lv[l];
      const int o = (int)off[l][p], oc = (int)off[l + 1][p];
      const int na = (int)S.aptr.size() - 1;
      for (int a = 0; a < na; ++a) {
        for (int m = S.aptr[a]; m < S.aptr[a + 1]; ++m) L.arows.push_back(S.arows[m] + o);
        L.aptr.push_back((int)L.arows.size());
        L.coff.push_back(oc + S.coff[a + 1]);
        if (ubase + S.uoff[a + 1] >= ((int64_t)1 << 31)) throw Error(-1, "batch too large for 32-bit block offsets");
        L.uoff.push_back((int)(ubase + S.uoff[a + 1]));
      }
      L.U.insert(L.U.end(), S.U.begin(), S.U.end());
      ubase += (int64_t)S.U.size();
    }
  }
  return U;
}

// ----------------------------------------------------------- device layout

constexpr int kKmax = 8;  // largest group / aggregate block handled by the kernels

struct Slab {
  int row0, nrows, width, off;  // sliced ELL: 64 rows, column-major entries
};

struct LevelLayout {
  int n = 0;
  bool sell = false;  // point groups stored as sliced ELL (64-row slabs)
  int G = 8;          // grouped CSR: kernel instantiation for groups of <= G rows
  int kmax = 1;
  std::vector<int> perm, iperm;  // new -> old, old -> new
  std::vector<int> gstart;       // ngroups + 1, rows in new numbering
  std::vector<int> sgrp;         // nstages + 1, group ranges of the stages
  // sliced ELL (sell) or grouped CSR (else) of the entries outside the diagonal blocks
  std::vector<Slab> slabs;
  std::vector<int> sslab;  // nstages + 1 slab ranges of the stages
  std::vector<int> rowptr;
  // grouped CSR: a row's entries in increasing column order; rsplit[p] is its
  // first entry in a later smoother stage (the forward sweep from x = 0 reads
  // only the entries before it)
  std::vector<int> rsplit;
  // grouped CSR, the index lists the kernels read: the rows of a group
  // usually share one column list (the Galerkin product couples whole
  // aggregates), stored once; otherwise the group's rows' lists follow each
  // other.  Entry e of row l (0-based in the group) of group g has its column
  // at gcol[e + gcsh[g] - l * gcm[g]] (gcm = the shared row length, or 0).
  std::vector<int> gcol, gcsh, gcm;
  bool all_shared = false;  // every group's rows share one list
  std::vector<int64_t> stage_gidx;       // per stage: stored column indices
  std::vector<int64_t> stage_later_idx;  // per stage: stored indices of later-stage columns
  std::vector<int> col;
  std::vector<double> val;
  std::vector<int> src;  // index of each entry in the file's CSR value array (-1: padding)
  // sliced ELL with 16-bit columns: slab s whose j-th entries span at most
  // 65535 columns stores them as col16[off + 64 j + i] = col - cbase[scb[s] + j]
  // (cbase padded to a multiple of 8 per slab); scb[s] = -1 keeps col.
  std::vector<uint16_t> col16;
  std::vector<int> cbase, scb;
  // col16 and vcode are stored lane-packed: the slots of entries j .. j + 7
  // (j a multiple of 8) of a slab's lane are adjacent, at pk_index(s, j, lane)
  // (one 16-byte / 8-byte load per lane for eight entries; positions past
  // the width up to a multiple of 8 hold delta 0 and code 0)
  std::vector<int> pk;
  int64_t nnz16 = 0;                // stored entries (without padding) in 16-bit slabs
  // sliced ELL with few distinct values: 1-byte codes into a table of at most
  // 256 values, for the entries (vcode, same positions as val) and for the
  // diagonal (dcode, one per row)
  bool vcoded = false, dcoded = false;
  std::vector<uint8_t> vcode, dcode;
  std::vector<double> vtab, dtab;
  std::vector<int64_t> stage_nnz16;  // the same per stage
  // dense k x k diagonal blocks of the groups (row-major)
  std::vector<int> dboff;
  std::vector<double> dblk;
  std::vector<int> dsrc;
};

inline int64_t pk_index(const LevelLayout& Y, int s, int j, int lane) {
  return (int64_t)Y.pk[s] + (int64_t)(j / 8) * 512 + lane * 8 + (j % 8);
}

struct TransferLayout {
  int nagg = 0, max_na = 0;
  std::vector<int> aptr, arows, uoff;
  std::vector<int> cst, kk;  // first coarse row (new numbering of the next level), block width
  std::vector<double> U;
};

// rowprob (optional, file-row order): the problem of every row when the
// level belongs to a batch; sliced-ELL slabs are then cut where it changes.
// 1-byte codes of v into a table of its distinct values (compared bit for
// bit), if there are at most 256 of them; false (code and tab cleared) if not.
inline bool encode_values(const std::vector<double>& v, std::vector<uint8_t>& code, std::vector<double>& tab) {
  code.clear();
  tab.clear();
  if (v.empty()) return false;
  std::vector<uint64_t> bits(v.size());
  std::memcpy(bits.data(), v.data(), v.size() * sizeof(double));
  std::vector<uint64_t> u(bits);
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  if (u.size() > 256) return false;
  tab.resize(u.size());
  std::memcpy(tab.data(), u.data(), u.size() * sizeof(double));
  code.resize(v.size());
  for (size_t i = 0; i < v.size(); ++i)
    code[i] = (uint8_t)(std::lower_bound(u.begin(), u.end(), bits[i]) - u.begin());
  return true;
}

inline void build_level_layout(const HostLevel& L, LevelLayout& Y, const std::vector<int>* rowprob = nullptr) {
  const int n = L.n;
  Y.n = n;
  if ((int)L.order.size() != n) throw Error(-2, "smoother order has wrong length");
  const int ng = (int)L.gptr.size() - 1;
  const int ns = (int)L.sptr.size() - 1;
  if (ng < 1 || L.gptr[0] != 0 || L.gptr[ng] != n || ns < 1 || L.sptr[0] != 0 || L.sptr[ns] != ng)
    throw Error(-2, "inconsistent smoother groups");
  for (int g = 0; g < ng; ++g)
    if (L.gptr[g + 1] <= L.gptr[g]) throw Error(-2, "empty smoother group");
  // Groups of one stage are mutually independent, so their order inside the
  // stage does not change the sweep.  On levels with multi-row groups they are
  // sorted by the aggregate (of the transfer to the next level) that holds
  // their first row, so the transfers read and write contiguous runs; on
  // point levels the file order is kept, which keeps the neighbour gathers of
  // the sliced-ELL products local (for a grid numbering).
  bool multi = false;
  for (int g = 0; g < ng; ++g) multi = multi || (L.gptr[g + 1] - L.gptr[g] > 1);
  std::vector<int> aggof(n, 0);
  for (int a = 0; a + 1 < (int)L.aptr.size(); ++a)
    for (int m = L.aptr[a]; m < L.aptr[a + 1]; ++m)
      if (L.arows[m] >= 0 && L.arows[m] < n) aggof[L.arows[m]] = a;
  std::vector<int> gorder(ng);
  for (int g = 0; g < ng; ++g) gorder[g] = g;
  for (int c = 0; c < ns && multi; ++c)
    std::stable_sort(gorder.begin() + L.sptr[c], gorder.begin() + L.sptr[c + 1], [&](int a, int b) {
      return aggof[L.order[L.gptr[a]]] < aggof[L.order[L.gptr[b]]];
    });
  Y.perm.clear();
  Y.perm.reserve(n);
  Y.gstart.assign(ng + 1, 0);
  for (int t = 0; t < ng; ++t) {
    const int g = gorder[t];
    for (int q = L.gptr[g]; q < L.gptr[g + 1]; ++q) Y.perm.push_back(L.order[q]);
    Y.gstart[t + 1] = (int)Y.perm.size();
  }
  Y.sgrp = L.sptr;
  Y.iperm.assign(n, -1);
  for (int p = 0; p < n; ++p) {
    const int i = Y.perm[p];
    if (i < 0 || i >= n || Y.iperm[i] >= 0) throw Error(-2, "smoother order is not a permutation");
    Y.iperm[i] = p;
  }
  std::vector<int> grp(n);
  Y.kmax = 1;
  bool point = true;
  for (int g = 0; g < ng; ++g) {
    const int k = Y.gstart[g + 1] - Y.gstart[g];
    if (k < 1) throw Error(-2, "empty smoother group");
    if (k > kKmax) throw Error(-1, "smoother group larger than 8 rows is not supported");
    Y.kmax = std::max(Y.kmax, k);
    if (k > 1) point = false;
    for (int p = Y.gstart[g]; p < Y.gstart[g + 1]; ++p) grp[p] = g;
    // rows of a group are consecutive in the file numbering as well
    for (int p = Y.gstart[g] + 1; p < Y.gstart[g + 1]; ++p)
      if (Y.perm[p] != Y.perm[p - 1] + 1) throw Error(-2, "smoother group rows not consecutive");
  }
  // stage independence: coupled rows of different groups lie in different stages
  std::vector<int> stage(ng);
  for (int c = 0; c < ns; ++c)
    for (int g = Y.sgrp[c]; g < Y.sgrp[c + 1]; ++g) stage[g] = c;
  Y.dboff.assign(ng + 1, 0);
  for (int g = 0; g < ng; ++g) {
    const int k = Y.gstart[g + 1] - Y.gstart[g];
    Y.dboff[g + 1] = Y.dboff[g] + k * k;
  }
  Y.dblk.assign(Y.dboff[ng], 0.0);
  Y.dsrc.assign(Y.dboff[ng], -1);
  int maxlen = 0;
  int64_t offcount = 0;
  for (int p = 0; p < n; ++p) {
    const int i = Y.perm[p], g = grp[p], g0 = Y.gstart[g], k = Y.gstart[g + 1] - g0;
    int len = 0;
    bool hasdiag = false;
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
      const int q = Y.iperm[L.ci[e]];
      if (q >= g0 && q < g0 + k) {
        const int idx = Y.dboff[g] + (p - g0) * k + (q - g0);
        Y.dblk[idx] += L.v[e];
        Y.dsrc[idx] = e;
        if (q == p) hasdiag = true;
      } else {
        if (stage[grp[q]] == stage[g]) throw Error(-2, "smoother stage couples two of its groups");
        ++len;
      }
    }
    if (!hasdiag) throw Error(-3, "missing diagonal entry");
    const double d = Y.dblk[Y.dboff[g] + (p - g0) * k + (p - g0)];
    if (!(d > 0.0)) throw Error(-3, "non-positive diagonal entry");
    maxlen = std::max(maxlen, len);
    offcount += len;
  }
  if (offcount > (int64_t)1 << 30) throw Error(-1, "level too large for 32-bit entry offsets");
  Y.sell = point && maxlen <= 64;
  if (Y.sell) {
    Y.sslab.assign(ns + 1, 0);
    for (int c = 0; c < ns; ++c) {
      const int r0 = Y.gstart[Y.sgrp[c]], r1 = Y.gstart[Y.sgrp[c + 1]];
      for (int b = r0; b < r1;) {
        Slab s;
        s.row0 = b;
        s.nrows = std::min(64, r1 - b);
        if (rowprob)
          for (int q = 1; q < s.nrows; ++q)
            if ((*rowprob)[Y.perm[b + q]] != (*rowprob)[Y.perm[b]]) {
              s.nrows = q;
              break;
            }
        s.width = 0;
        for (int p = b; p < b + s.nrows; ++p) {
          const int i = Y.perm[p];
          s.width = std::max(s.width, L.rp[i + 1] - L.rp[i] - 1);
        }
        s.off = 0;
        Y.slabs.push_back(s);
        b += s.nrows;
      }
      Y.sslab[c + 1] = (int)Y.slabs.size();
    }
    int64_t tot = 0;
    for (Slab& s : Y.slabs) {
      s.off = (int)tot;
      tot += (int64_t)s.width * 64;
      if (tot > ((int64_t)1 << 31) - 1) throw Error(-1, "level too large for 32-bit slab offsets");
    }
    Y.col.assign(tot, 0);
    Y.val.assign(tot, 0.0);
    Y.src.assign(tot, -1);
    for (const Slab& s : Y.slabs)
      for (int lane = 0; lane < s.nrows; ++lane) {
        const int p = s.row0 + lane, i = Y.perm[p];
        int j = 0;
        for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
          const int q = Y.iperm[L.ci[e]];
          if (q == p) continue;
          const int64_t at = (int64_t)s.off + (int64_t)j * 64 + lane;
          Y.col[at] = q;
          Y.val[at] = L.v[e];
          Y.src[at] = e;
          ++j;
        }
        for (; j < s.width; ++j) Y.col[(int64_t)s.off + (int64_t)j * 64 + lane] = p;  // zero padding
      }
    // 16-bit column deltas per (slab, entry position) where they fit
    Y.col16.assign(tot, 0);
    Y.scb.assign(Y.slabs.size(), -1);
    Y.cbase.clear();
    Y.nnz16 = 0;
    Y.stage_nnz16.assign(ns, 0);
    std::vector<int> slab_stage(Y.slabs.size());
    for (int c = 0; c < ns; ++c)
      for (int q = Y.sslab[c]; q < Y.sslab[c + 1]; ++q) slab_stage[q] = c;
    for (size_t q = 0; q < Y.slabs.size(); ++q) {
      const Slab& s = Y.slabs[q];
      std::vector<int> lo(s.width, INT32_MAX), hi(s.width, INT32_MIN);
      int64_t real = 0;
      for (int lane = 0; lane < s.nrows; ++lane) {
        const int i = Y.perm[s.row0 + lane];
        const int len = L.rp[i + 1] - L.rp[i] - 1;
        real += len;
        for (int j = 0; j < len; ++j) {
          const int c = Y.col[(int64_t)s.off + (int64_t)j * 64 + lane];
          lo[j] = std::min(lo[j], c);
          hi[j] = std::max(hi[j], c);
        }
      }
      bool fits = true;
      for (int j = 0; j < s.width; ++j) {
        if (lo[j] > hi[j]) lo[j] = hi[j] = s.row0;  // only padding in this position
        fits = fits && (int64_t)hi[j] - lo[j] <= 65535;
      }
      if (!fits) continue;
      Y.scb[q] = (int)Y.cbase.size();
      const int wpad = (s.width + 7) / 8 * 8;
      for (int j = 0; j < wpad; ++j) Y.cbase.push_back(lo[std::min(j, s.width - 1)]);
      for (int lane = 0; lane < s.nrows; ++lane)
        for (int j = 0; j < s.width; ++j) {
          const int64_t at = (int64_t)s.off + (int64_t)j * 64 + lane;
          const int64_t d = (int64_t)Y.col[at] - lo[j];
          // padding (value 0) whose own row is out of range points at the base
          Y.col16[at] = (uint16_t)((d >= 0 && d <= 65535) ? d : 0);
        }
      Y.nnz16 += real;
      Y.stage_nnz16[slab_stage[q]] += real;
    }
    // value dictionaries: where a sliced-ELL level's entries (or its
    // diagonal) take at most 256 distinct values, the kernels read 1-byte
    // codes and look the values up (exact: the same binary64 values)
    Y.vcoded = encode_values(Y.val, Y.vcode, Y.vtab);
    Y.dcoded = encode_values(Y.dblk, Y.dcode, Y.dtab);
    // lane-packed copies of the 16-bit deltas and the codes
    Y.pk.assign(Y.slabs.size(), 0);
    int64_t tp = 0;
    for (size_t q = 0; q < Y.slabs.size(); ++q) {
      Y.pk[q] = (int)tp;
      tp += (int64_t)(Y.slabs[q].width + 7) / 8 * 512;
      if (tp > ((int64_t)1 << 31) - 1) throw Error(-1, "level too large for 32-bit packed offsets");
    }
    std::vector<uint16_t> c16p(tp, 0);
    std::vector<uint8_t> vcp(Y.vcoded ? tp : 0, 0);
    for (size_t q = 0; q < Y.slabs.size(); ++q) {
      const Slab& sl = Y.slabs[q];
      for (int j = 0; j < sl.width; ++j)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t at = (int64_t)sl.off + (int64_t)j * 64 + lane, to = pk_index(Y, (int)q, j, lane);
          c16p[to] = Y.col16[at];
          if (Y.vcoded) vcp[to] = Y.vcode[at];
        }
    }
    Y.col16.swap(c16p);
    if (Y.vcoded) Y.vcode.swap(vcp);
  } else {
    Y.rowptr.assign(n + 1, 0);
    Y.rsplit.assign(n, 0);
    Y.col.reserve(offcount);
    Y.val.reserve(offcount);
    Y.src.reserve(offcount);
    // The rows of a group whose column lists differ only a little (a few
    // structurally zero couplings) are padded with explicit zeros (src -1) to
    // the union of their lists, so that they share one list: at most a
    // quarter more stored values.
    std::vector<std::vector<int>> ents(kKmax);
    std::vector<int> uni;
    const int ngr = (int)Y.gstart.size() - 1;
    for (int g = 0; g < ngr; ++g) {
      const int g0 = Y.gstart[g], k = Y.gstart[g + 1] - g0;
      const int later = Y.gstart[Y.sgrp[stage[g] + 1]];  // first row of the next stage
      int64_t own = 0;
      uni.clear();
      for (int l = 0; l < k; ++l) {
        const int i = Y.perm[g0 + l];
        std::vector<int>& el = ents[l];
        el.clear();
        for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
          const int q = Y.iperm[L.ci[e]];
          if (q < g0 || q >= g0 + k) el.push_back(e);
        }
        std::sort(el.begin(), el.end(), [&](int a, int b) { return Y.iperm[L.ci[a]] < Y.iperm[L.ci[b]]; });
        own += (int64_t)el.size();
        for (int e : el) uni.push_back(Y.iperm[L.ci[e]]);
      }
      std::sort(uni.begin(), uni.end());
      uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
      const bool pad = k > 1 && 4 * (int64_t)k * (int64_t)uni.size() <= 5 * own;
      for (int l = 0; l < k; ++l) {
        const int p = g0 + l;
        Y.rsplit[p] = (int)Y.col.size();
        size_t t = 0;
        const std::vector<int>& el = ents[l];
        const size_t len = pad ? uni.size() : el.size();
        for (size_t u = 0; u < len; ++u) {
          int q, e = -1;
          if (pad) {
            q = uni[u];
            if (t < el.size() && Y.iperm[L.ci[el[t]]] == q) e = el[t++];
          } else {
            e = el[u];
            q = Y.iperm[L.ci[e]];
          }
          Y.col.push_back(q);
          Y.val.push_back(e >= 0 ? L.v[e] : 0.0);
          Y.src.push_back(e);
          if (q < later) Y.rsplit[p] = (int)Y.col.size();
        }
        Y.rowptr[p + 1] = (int)Y.col.size();
      }
    }
    // shared column lists
    const int ng = (int)Y.gstart.size() - 1, ns = (int)Y.sgrp.size() - 1;
    Y.gcsh.assign(ng, 0);
    Y.gcm.assign(ng, 0);
    Y.all_shared = true;
    Y.gcol.clear();
    Y.stage_gidx.assign(ns, 0);
    Y.stage_later_idx.assign(ns, 0);
    for (int c = 0; c < ns; ++c)
      for (int g = Y.sgrp[c]; g < Y.sgrp[c + 1]; ++g) {
        const int p0 = Y.gstart[g], k = Y.gstart[g + 1] - p0, e0 = Y.rowptr[p0], m = Y.rowptr[p0 + 1] - e0;
        bool shared = true;
        for (int l = 1; l < k && shared; ++l) {
          const int el = Y.rowptr[p0 + l];
          shared = Y.rowptr[p0 + l + 1] - el == m && Y.rsplit[p0 + l] - el == Y.rsplit[p0] - e0 &&
                   std::equal(Y.col.begin() + el, Y.col.begin() + el + m, Y.col.begin() + e0);
        }
        const int at = (int)Y.gcol.size();
        const int e1 = shared ? e0 + m : Y.rowptr[p0 + k];
        Y.gcol.insert(Y.gcol.end(), Y.col.begin() + e0, Y.col.begin() + e1);
        Y.gcsh[g] = at - e0;
        Y.gcm[g] = shared ? m : 0;
        Y.all_shared = Y.all_shared && shared;
        Y.stage_gidx[c] += e1 - e0;
        if (shared)
          Y.stage_later_idx[c] += Y.rowptr[p0 + 1] - Y.rsplit[p0];
        else
          for (int l = 0; l < k; ++l) Y.stage_later_idx[c] += Y.rowptr[p0 + l + 1] - Y.rsplit[p0 + l];
      }
    // kernels are instantiated for groups of up to 1, 2, 4 or 8 rows
    Y.G = Y.kmax <= 1 ? 1 : Y.kmax <= 2 ? 2 : Y.kmax <= 4 ? 4 : 8;
  }
}

inline void build_transfer_layout(const HostLevel& L, const LevelLayout& Yf, const LevelLayout* Yc,
                                  TransferLayout& T) {
  const int na = (int)L.aptr.size() - 1;
  T.nagg = na;
  T.aptr = L.aptr;
  T.uoff = L.uoff;
  // U_a stored column-major (k_a x n_a): column l of a block is one
  // contiguous, coalesced run for the wave that handles the aggregate.  The
  // members of an aggregate are listed in increasing level order (the order
  // of the file's members is immaterial to P), so the members of earlier
  // smoother stages come first and the U entries of later stages' members
  // share no cache line with them.
  T.U.resize(L.U.size());
  T.arows.resize(L.arows.size());
  std::vector<int> ord;
  for (int a = 0; a < na; ++a) {
    const int m = L.aptr[a + 1] - L.aptr[a], k = L.coff[a + 1] - L.coff[a], m0 = L.aptr[a];
    ord.resize(m);
    for (int li = 0; li < m; ++li) ord[li] = li;
    std::sort(ord.begin(), ord.end(),
              [&](int x, int y) { return Yf.iperm[L.arows[m0 + x]] < Yf.iperm[L.arows[m0 + y]]; });
    for (int t = 0; t < m; ++t) {
      const int li = ord[t];
      T.arows[m0 + t] = Yf.iperm[L.arows[m0 + li]];
      for (int l = 0; l < k; ++l) T.U[(size_t)L.uoff[a] + (size_t)l * m + t] = L.U[(size_t)L.uoff[a] + (size_t)li * k + l];
    }
  }
  T.cst.resize(na);
  T.kk.resize(na);
  T.max_na = 0;
  for (int a = 0; a < na; ++a) {
    const int k = L.coff[a + 1] - L.coff[a];
    if (k > kKmax) throw Error(-1, "aggregate basis wider than 8 columns is not supported");
    T.kk[a] = k;
    T.max_na = std::max(T.max_na, L.aptr[a + 1] - L.aptr[a]);
    if (Yc) {
      T.cst[a] = Yc->iperm[L.coff[a]];
      for (int l = 1; l < k; ++l)
        if (Yc->iperm[L.coff[a] + l] != T.cst[a] + l)
          throw Error(-2, "coarse dofs of an aggregate are not a smoother group");
    } else {
      T.cst[a] = L.coff[a];
    }
  }
}

}  // namespace mvamg
