// Host side of libfctn.so: descriptor validation, workspace carving, the
// per-mode operand tables, the sweep scheduler (Algorithms 1-2, including the
// pair-tensor cache of the reuse mechanism and the alternating factor order),
// the continuous-batching server and the C ABI declared in fctn.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fctn.h"
#include "kernels.hpp"

using namespace fctn;

namespace {

constexpr int kHist = 4096;
constexpr int kTargetGramWGs = 512;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad16(int x) { return (x + 15) / 16 * 16; }

struct Carver {
  char* base;
  size_t off;
  void* take(size_t bytes) {
    off = align256(off);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

enum Src { SRC_F0 = 0, SRC_P12 = 10, SRC_P34 = 11, SRC_GRP = 16 };

// orders N >= 5: the prefix groups A_1..A_j (j = 2 .. N-2) and the suffix
// groups A_j..A_N (j = 3 .. N-1), 1-based, each one factor more than its
// parent group
constexpr int kMaxGroups = 2 * (FCTN_MAX_ORDER - 3);

struct ModeInfo {
  int64_t Ik, s, C, spost;
  int u_src, v_src;
  MGen mg;          // strides/sizes; U/V pointers resolved at launch
  XView xv;
  GramGeom geom;
  RecGeom rg;
  int ncls;
};

// one cached group of the general-order chain: members[0] (x) members[1]
// contracted over their shared bonds
struct GroupSlot {
  GroupDesc gd;       // member pointers are filled at launch
  int src[2];         // SRC_F0 + factor or SRC_GRP + group
  uint32_t fmask;     // factors contracted into the group
  int64_t num;        // entries
  void* buf;
  bool built;
  int64_t snap[FCTN_MAX_ORDER];   // factor versions it was built from
};

struct ProfRec {
  int stage;
  hipEvent_t a, b;
  double flops, bytes;
};

struct ProfState {
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
};

}  // namespace

struct fctn_plan_s {
  fctn_desc d;
  int N, prec;
  int64_t dims[FCTN_MAX_ORDER];
  int R[FCTN_MAX_ORDER][FCTN_MAX_ORDER];
  int64_t numel;
  size_t es;         // bytes per X element
  hipStream_t st;
  void* X;
  void* Z;
  uint32_t* bits;
  int32_t* bad_part;
  int32_t* bad_flag;
  int32_t* dev_err;  // set by a kernel whose bounded wait gave up
  int bad_nblk;
  double* A64[FCTN_MAX_ORDER];
  void* Aw[FCTN_MAX_ORDER];
  void* Au[FCTN_MAX_ORDER];
  int64_t fnum[FCTN_MAX_ORDER];
  void* P[2];
  int64_t pnum[2];
  GroupDesc pgd[2];
  void* part;
  void* part_cur;    // where this call's split-K partials go: part, or the
                     // static scratch array (fctn_sweep_noalloc)
  double *G, *B, *At;
  double* Q[FCTN_MAX_ORDER];
  double* Qt[FCTN_MAX_ORDER];
  double* lamcol[FCTN_MAX_ORDER];
  double* trace_part;
  int max_cls;
  size_t part_bytes;  // size of the split-K partial region
  double* lam_half;
  int32_t* ncls_dev;
  double* xpart;
  int xblocks;      // blocks of the X update (one partial triple each)
  double* hist;
  double* scratch_slot;
  ModeInfo mode[FCTN_MAX_ORDER];
  GroupSlot grp[kMaxGroups];   // orders N >= 5
  int ngrp;
  int64_t sweeps_done;
  int64_t hist_first;  // first sweep index whose history this plan holds
  int64_t fver[FCTN_MAX_ORDER];
  int64_t pver[2][2];
  bool pvalid[2];
  fctn_status sticky;
  bool debug;
  bool prof_on;
  ProfState* prof;
};

namespace {

fctn_status validate(const fctn_desc* d) {
  if (!d) return FCTN_E_INVALID;
  if (d->order < 2 || d->order > FCTN_MAX_ORDER) return FCTN_E_INVALID;
  const int N = d->order;
  for (int k = 0; k < N; ++k) {
    if (d->dims[k] < 1) return FCTN_E_INVALID;
    if (!(d->lambda[k] >= 0.0) || !(d->delta[k] >= 0.0)) return FCTN_E_INVALID;
  }
  for (int b = 0; b < N * (N - 1) / 2; ++b)
    if (d->ranks[b] < 1) return FCTN_E_INVALID;
  if (!(d->rho > 0.0)) return FCTN_E_INVALID;
  if (d->precision < FCTN_F64 || d->precision > FCTN_BF16X3) return FCTN_E_INVALID;
  if (d->reuse != 0 && d->reuse != 1) return FCTN_E_INVALID;
  if (d->order_policy != 0 && d->order_policy != 1) return FCTN_E_INVALID;
  if (!(d->extrap_alpha >= 0.0 && d->extrap_alpha < 1.0)) return FCTN_E_INVALID;
  if (!(d->extrap_beta >= 0.0 && d->extrap_beta <= 1.0)) return FCTN_E_INVALID;
  if (N < 3) return FCTN_E_UNSUPPORTED;
  return FCTN_OK;
}

void fill_ranks(const fctn_desc* d, int R[FCTN_MAX_ORDER][FCTN_MAX_ORDER]) {
  const int N = d->order;
  int b = 0;
  for (int i = 0; i < N; ++i) {
    R[i][i] = 0;
    for (int j = i + 1; j < N; ++j) {
      R[i][j] = R[j][i] = d->ranks[b++];
    }
  }
}

// Orders N >= 5 (Algorithm 2's reuse, Section 3.4, Table 2).  For mode k the
// other factors split into two runs of consecutive modes, U below V:
//   k = 1, 2:        U = {A_{3-k}},       V = A_3..A_N
//   3 <= k <= N-1:   U = A_1..A_{k-1},    V = A_{k+1}..A_N
//   k = N:           U = A_1..A_{N-2},    V = {A_{N-1}}
// (1-based), so that the columns (i_U, i_V) of M_k are a strided view of X
// and the rows (bonds to k from U, then from V) follow A_k's bond order.  A
// run of one factor is read in place; a longer run is a cached group: the
// prefix A_1..A_j is built as (A_1..A_{j-1}) (x) A_j and the suffix A_j..A_N
// as A_j (x) (A_{j+1}..A_N), and a group is rebuilt only when one of its
// factors has changed since it was built.  In the fixed order 1..N a sweep
// builds one pair and N-4 larger groups on each side.
//
// Layouts are lists of keys, the last fastest: a key is a physical index
// (a == b) or a bond {a < b}.
//   factor f:  for l = 0..N-1: l == f ? i_f : bond(f, l)          (0-based)
//   prefix j:  i_0..i_j | bond(s, j+1), s = 0..j | bond(s, t), s = 0..j, t = j+2..N-1
//   suffix j:  i_j..i_{N-1} | bond(t, s), s = 0..j-1, t = j..N-1
// The prefix keeps the bonds to the next factor as one block (the rows of M
// for mode j+1, the internal bonds of the next prefix), the suffix its bonds
// grouped by the outside factor, so that every block M_k or a chain step
// reads is a run of consecutive keys.
struct Key {
  int a, b;
  int64_t size;
};
typedef std::vector<Key> Layout;

Key phys_key(const fctn_plan_s* P, int l) { return Key{l, l, P->dims[l]}; }
Key bond_key(const fctn_plan_s* P, int s, int t) {
  return Key{std::min(s, t), std::max(s, t), P->R[s][t]};
}

Layout factor_layout(const fctn_plan_s* P, int f) {
  Layout L;
  for (int l = 0; l < P->N; ++l) L.push_back(l == f ? phys_key(P, f) : bond_key(P, f, l));
  return L;
}

Layout prefix_layout(const fctn_plan_s* P, int j) {
  Layout L;
  for (int l = 0; l <= j; ++l) L.push_back(phys_key(P, l));
  for (int s = 0; s <= j; ++s) L.push_back(bond_key(P, s, j + 1));
  for (int s = 0; s <= j; ++s)
    for (int t = j + 2; t < P->N; ++t) L.push_back(bond_key(P, s, t));
  return L;
}

Layout suffix_layout(const fctn_plan_s* P, int j) {
  Layout L;
  for (int l = j; l < P->N; ++l) L.push_back(phys_key(P, l));
  for (int s = 0; s < j; ++s)
    for (int t = j; t < P->N; ++t) L.push_back(bond_key(P, t, s));
  return L;
}

int find_key(const Layout& L, const Key& k) {
  for (size_t i = 0; i < L.size(); ++i)
    if (L[i].a == k.a && L[i].b == k.b) return (int)i;
  return -1;
}

int64_t key_stride(const Layout& L, int i) {
  int64_t st = 1;
  for (size_t l = i + 1; l < L.size(); ++l) st *= L[l].size;
  return st;
}

int64_t layout_numel(const Layout& L) {
  int64_t n = 1;
  for (const Key& k : L) n *= k.size;
  return n;
}

// the keys sit in L consecutively and in this order: their flat index has
// the stride of the last one
bool block_stride(const Layout& L, const std::vector<Key>& keys, int64_t* st, int64_t* size) {
  if (keys.empty()) return false;
  const int i0 = find_key(L, keys[0]);
  if (i0 < 0 || i0 + keys.size() > L.size()) return false;
  *size = 1;
  for (size_t q = 0; q < keys.size(); ++q) {
    if (L[i0 + q].a != keys[q].a || L[i0 + q].b != keys[q].b) return false;
    *size *= keys[q].size;
  }
  *st = key_stride(L, i0 + (int)keys.size() - 1);
  return true;
}

// launch shape of the contraction kernel: the inner block is the smallest
// run of trailing output digits with at least 256 entries (four a lane)
// whose member rows fit the LDS budget; short blocks share a pass of at
// least 256 entries
bool group_launch_shape(GroupDesc* gd, size_t es) {
  const int64_t ip = (gd->inner + 3) / 4 * 4;
  auto lds = [&](int64_t sin, int64_t s0, int64_t s1, int64_t no) {
    return (int64_t)es * no * (s0 + s1) * ip + 4 * (sin + s0 + s1 + 2 * ip + 2 * no);
  };
  int ds = gd->nd;
  int64_t sin = 1, s0 = 1, s1 = 1, bs = 1, b0 = 1, b1 = 1;
  for (int d = gd->nd - 1; d >= 0; --d) {
    sin *= gd->dsize[d];
    (gd->dmem[d] == 0 ? s0 : s1) *= gd->dsize[d];
    if (sin > 4096 || lds(sin, s0, s1, 1) > kGroupMaxLds) break;
    ds = d;
    bs = sin;
    b0 = s0;
    b1 = s1;
    if (sin >= 256) break;
  }
  int64_t no = std::max<int64_t>(1, (256 + bs - 1) / bs);
  while (no > 1 && lds(bs, b0, b1, no) > kGroupMaxLds) --no;
  if (lds(bs, b0, b1, no) > kGroupMaxLds) return false;
  gd->ds = ds;
  gd->sin = (int32_t)bs;
  gd->sin0 = (int32_t)b0;
  gd->sin1 = (int32_t)b1;
  gd->innerp = (int32_t)ip;
  gd->no = (int32_t)no;
  gd->nouter = (int32_t)(gd->total / bs);
  gd->lds_bytes = (int32_t)lds(bs, b0, b1, no);
  for (int d = ds; d < gd->nd; ++d) gd->m_dsize[d] = div_magic((uint32_t)gd->dsize[d]);
  gd->m_ip = div_magic((uint32_t)ip);
  gd->m_n0 = div_magic((uint32_t)b0);
  gd->m_n1 = div_magic((uint32_t)b1);
  gd->m_nin = div_magic((uint32_t)bs);
  // the quotients formed with these multipliers stay below 2^16
  return no * (b0 + b1) * ip < 65536 && no * bs < 65536;
}

// GroupDesc of out = m0 (x) m1, contracted over the keys both members hold;
// every offset the kernel forms is checked against the member sizes
bool chain_desc(const Layout& m0, const Layout& m1, const Layout& out, size_t es,
                GroupDesc* gd) {
  memset(gd, 0, sizeof(*gd));
  const Layout* M[2] = {&m0, &m1};
  std::vector<int64_t> dsz, dmem, dst;
  for (size_t i = 0; i < out.size(); ++i) {
    const int i0 = find_key(m0, out[i]), i1 = find_key(m1, out[i]);
    if ((i0 >= 0) == (i1 >= 0)) return false;   // an output key is in exactly one member
    const int a = i0 >= 0 ? 0 : 1;
    const int64_t st = key_stride(*M[a], a == 0 ? i0 : i1);
    const int64_t sz = out[i].size;
    if (!dsz.empty() && dmem.back() == a && dst.back() == st * sz) {
      dsz.back() *= sz;        // merge with the slower digit
      dst.back() = st;
    } else {
      dsz.push_back(sz);
      dmem.push_back(a);
      dst.push_back(st);
    }
  }
  std::vector<int64_t> isz, ist0, ist1;
  for (size_t i = 0; i < m0.size(); ++i) {
    if (find_key(out, m0[i]) >= 0) continue;
    const int i1 = find_key(m1, m0[i]);
    if (i1 < 0) return false;                      // summed in one member only
    const int64_t s0 = key_stride(m0, (int)i), s1 = key_stride(m1, i1), sz = m0[i].size;
    if (!isz.empty() && ist0.back() == s0 * sz && ist1.back() == s1 * sz) {
      isz.back() *= sz;
      ist0.back() = s0;
      ist1.back() = s1;
    } else {
      isz.push_back(sz);
      ist0.push_back(s0);
      ist1.push_back(s1);
    }
  }
  for (const Key& k : m1)
    if (find_key(out, k) < 0 && find_key(m0, k) < 0) return false;
  if (dsz.size() > (size_t)kGroupMaxDigits || isz.size() > (size_t)kGroupMaxDigits) return false;
  int64_t mx[2] = {0, 0}, inner = 1;
  for (size_t d = 0; d < dsz.size(); ++d) {
    gd->dsize[d] = (int32_t)dsz[d];
    gd->dmem[d] = (int32_t)dmem[d];
    gd->dstr[d] = (int32_t)dst[d];
    mx[dmem[d]] += (dsz[d] - 1) * dst[d];
  }
  for (size_t i = 0; i < isz.size(); ++i) {
    gd->isize[i] = (int32_t)isz[i];
    gd->istr0[i] = (int32_t)ist0[i];
    gd->istr1[i] = (int32_t)ist1[i];
    mx[0] += (isz[i] - 1) * ist0[i];
    mx[1] += (isz[i] - 1) * ist1[i];
    inner *= isz[i];
  }
  gd->nd = (int32_t)dsz.size();
  gd->ni = (int32_t)isz.size();
  const int64_t total = layout_numel(out);
  if (total >= ((int64_t)1 << 31) || inner > kGroupMaxInner) return false;
  for (int a = 0; a < 2; ++a)
    if (mx[a] >= layout_numel(*M[a]) || layout_numel(*M[a]) >= ((int64_t)1 << 31)) return false;
  gd->total = (int32_t)total;
  gd->inner = (int32_t)inner;
  return group_launch_shape(gd, es);
}

int prefix_gid(int j) { return j - 1; }                  // j = 1 .. N-3 (0-based)
int suffix_gid(int N, int j) { return (N - 3) + (j - 2); }  // j = 2 .. N-2

// the operand of consecutive modes lo..hi: a factor, a prefix or a suffix
bool run_operand(const fctn_plan_s* P, int lo, int hi, int* src, Layout* L) {
  const int N = P->N;
  if (lo == hi) {
    *src = SRC_F0 + lo;
    *L = factor_layout(P, lo);
  } else if (lo == 0 && hi >= 1 && hi <= N - 3) {
    *src = SRC_GRP + prefix_gid(hi);
    *L = prefix_layout(P, hi);
  } else if (hi == N - 1 && lo >= 2 && lo <= N - 2) {
    *src = SRC_GRP + suffix_gid(N, lo);
    *L = suffix_layout(P, lo);
  } else {
    return false;
  }
  return true;
}

bool setup_groups(fctn_plan_s* P) {
  const int N = P->N;
  P->ngrp = 2 * (N - 3);
  for (int j = 1; j <= N - 3; ++j) {             // prefixes, each from the previous
    GroupSlot& G = P->grp[prefix_gid(j)];
    Layout m0 = j == 1 ? factor_layout(P, 0) : prefix_layout(P, j - 1);
    G.src[0] = j == 1 ? SRC_F0 + 0 : SRC_GRP + prefix_gid(j - 1);
    G.src[1] = SRC_F0 + j;
    G.fmask = (2u << j) - 1;
    const Layout out = prefix_layout(P, j);
    if (!chain_desc(m0, factor_layout(P, j), out, P->es, &G.gd)) return false;
    G.num = layout_numel(out);
  }
  for (int j = N - 2; j >= 2; --j) {              // suffixes, each from the next
    GroupSlot& G = P->grp[suffix_gid(N, j)];
    Layout m1 = j == N - 2 ? factor_layout(P, N - 1) : suffix_layout(P, j + 1);
    G.src[0] = SRC_F0 + j;
    G.src[1] = j == N - 2 ? SRC_F0 + N - 1 : SRC_GRP + suffix_gid(N, j + 1);
    G.fmask = ((1u << N) - 1) & ~((1u << j) - 1);
    const Layout out = suffix_layout(P, j);
    if (!chain_desc(factor_layout(P, j), m1, out, P->es, &G.gd)) return false;
    G.num = layout_numel(out);
  }
  return true;
}

// MGen strides of one operand: rows (its bonds to k), columns (its physical
// indices) and kap (the bonds to the other operand, in `kap` order) must each
// be a run of consecutive keys of its layout, and nothing else may be in it
bool operand_strides(const Layout& L, const std::vector<Key>& rows, const std::vector<Key>& cols,
                     const std::vector<Key>& kap, int64_t* r_st, int64_t* c_st, int64_t* k_st,
                     int64_t* R, int64_t* C, int64_t* K) {
  if (L.size() != rows.size() + cols.size() + kap.size()) return false;
  return block_stride(L, rows, r_st, R) && block_stride(L, cols, c_st, C) &&
         block_stride(L, kap, k_st, K);
}

bool setup_mode_general(fctn_plan_s* P, int k) {
  const int N = P->N;
  const int64_t* I = P->dims;
  ModeInfo& m = P->mode[k];
  MGen& g = m.mg;
  XView& x = m.xv;
  int ulo, uhi, vlo, vhi;
  if (k <= 1) {
    ulo = uhi = 1 - k;
    vlo = 2;
    vhi = N - 1;
  } else if (k <= N - 2) {
    ulo = 0;
    uhi = k - 1;
    vlo = k + 1;
    vhi = N - 1;
  } else {
    ulo = 0;
    uhi = N - 3;
    vlo = vhi = N - 2;
  }
  Layout LU, LV;
  if (!run_operand(P, ulo, uhi, &m.u_src, &LU) || !run_operand(P, vlo, vhi, &m.v_src, &LV))
    return false;
  std::vector<Key> ru, cu, rv, cv, kap;
  for (int u = ulo; u <= uhi; ++u) {
    ru.push_back(bond_key(P, u, k));
    cu.push_back(phys_key(P, u));
  }
  for (int v = vlo; v <= vhi; ++v) {
    rv.push_back(bond_key(P, v, k));
    cv.push_back(phys_key(P, v));
  }
  for (const Key& key : LU)
    if (key.a != key.b) {
      const int o = key.a >= ulo && key.a <= uhi ? key.b : key.a;
      if (o >= vlo && o <= vhi) kap.push_back(key);
    }
  int64_t Ru, Cu, Ku, Rv, Cv, Kv;
  if (!operand_strides(LU, ru, cu, kap, &g.u_ru, &g.u_cu, &g.u_k, &Ru, &Cu, &Ku) ||
      !operand_strides(LV, rv, cv, kap, &g.v_rv, &g.v_cv, &g.v_k, &Rv, &Cv, &Kv))
    return false;
  if (Ku != Kv || Ru * Rv != m.s || Ku >= ((int64_t)1 << 31)) return false;
  g.Ru = (int32_t)Ru;
  g.Rv = (int32_t)Rv;
  g.K = (int32_t)Ku;
  g.Cu = Cu;
  g.Cv = Cv;
  auto xstride = [&](int l) {
    int64_t st = 1;
    for (int q = l + 1; q < N; ++q) st *= I[q];
    return st;
  };
  x.x_cu = xstride(uhi);
  x.x_cv = xstride(vhi);
  x.x_ik = xstride(k);
  return true;
}

// Operand tables: M_k[ru * Rv + rv, cu * Cv + cv] = sum U[ru, cu, kap] V[rv, cv, kap]
// where rows follow A_k's bond modes in order (last fastest) and columns the
// other physical modes in order (last fastest); see the derivation per mode.
bool setup_modes(fctn_plan_s* P) {
  const int N = P->N;
  const int64_t* I = P->dims;
  int(*R)[FCTN_MAX_ORDER] = P->R;
  if (N >= 5 && !setup_groups(P)) return false;
  for (int k = 0; k < N; ++k) {
    ModeInfo& m = P->mode[k];
    m.Ik = I[k];
    int64_t s = 1, spost = 1;
    for (int j = 0; j < N; ++j)
      if (j != k) s *= R[k][j];
    for (int j = k + 1; j < N; ++j) spost *= R[k][j];
    m.s = s;
    m.spost = spost;
    m.C = P->numel / I[k];
    m.ncls = (int)(I[k] / 2 + 1);
    MGen& g = m.mg;
    XView& x = m.xv;
    x.Ik = (int32_t)I[k];
    if (N >= 5) {
      if (!setup_mode_general(P, k)) return false;
    } else if (N == 3) {
      const int64_t I1 = I[0], I2 = I[1], I3 = I[2];
      const int64_t R12 = R[0][1], R13 = R[0][2], R23 = R[1][2];
      if (k == 0) {
        m.u_src = SRC_F0 + 1; g.u_ru = I2 * R23; g.u_cu = R23; g.u_k = 1; g.Ru = (int)R12; g.K = (int)R23;
        m.v_src = SRC_F0 + 2; g.v_rv = R23 * I3; g.v_cv = 1; g.v_k = I3; g.Rv = (int)R13;
        g.Cu = I2; g.Cv = I3; x.x_cu = I3; x.x_cv = 1; x.x_ik = I2 * I3;
      } else if (k == 1) {
        m.u_src = SRC_F0 + 0; g.u_ru = R13; g.u_cu = R12 * R13; g.u_k = 1; g.Ru = (int)R12; g.K = (int)R13;
        m.v_src = SRC_F0 + 2; g.v_rv = I3; g.v_cv = 1; g.v_k = R23 * I3; g.Rv = (int)R23;
        g.Cu = I1; g.Cv = I3; x.x_cu = I2 * I3; x.x_cv = 1; x.x_ik = I3;
      } else {
        m.u_src = SRC_F0 + 0; g.u_ru = 1; g.u_cu = R12 * R13; g.u_k = R13; g.Ru = (int)R13; g.K = (int)R12;
        m.v_src = SRC_F0 + 1; g.v_rv = 1; g.v_cv = R23; g.v_k = I2 * R23; g.Rv = (int)R23;
        g.Cu = I1; g.Cv = I2; x.x_cu = I2 * I3; x.x_cv = I3; x.x_ik = 1;
      }
    } else {
      const int64_t I1 = I[0], I2 = I[1], I3 = I[2], I4 = I[3];
      const int64_t R12 = R[0][1], R13 = R[0][2], R14 = R[0][3];
      const int64_t R23 = R[1][2], R24 = R[1][3], R34 = R[2][3];
      const int64_t pb = R13 * R14 * R23 * R24;   // bond block of either pair tensor
      if (k == 0) {
        m.u_src = SRC_F0 + 1; g.u_ru = I2 * R23 * R24; g.u_cu = R23 * R24; g.u_k = 1;
        g.Ru = (int)R12; g.K = (int)(R23 * R24);
        m.v_src = SRC_P34; g.v_rv = R23 * R24; g.v_cv = pb; g.v_k = 1; g.Rv = (int)(R13 * R14);
        g.Cu = I2; g.Cv = I3 * I4; x.x_cu = I3 * I4; x.x_cv = 1; x.x_ik = I2 * I3 * I4;
      } else if (k == 1) {
        m.u_src = SRC_F0 + 0; g.u_ru = R13 * R14; g.u_cu = R12 * R13 * R14; g.u_k = 1;
        g.Ru = (int)R12; g.K = (int)(R13 * R14);
        m.v_src = SRC_P34; g.v_rv = 1; g.v_cv = pb; g.v_k = R23 * R24; g.Rv = (int)(R23 * R24);
        g.Cu = I1; g.Cv = I3 * I4; x.x_cu = I2 * I3 * I4; x.x_cv = 1; x.x_ik = I3 * I4;
      } else if (k == 2) {
        m.u_src = SRC_P12; g.u_ru = R14 * R24; g.u_cu = pb; g.u_k = 1;
        g.Ru = (int)(R13 * R23); g.K = (int)(R14 * R24);
        m.v_src = SRC_F0 + 3; g.v_rv = I4; g.v_cv = 1; g.v_k = R34 * I4; g.Rv = (int)R34;
        g.Cu = I1 * I2; g.Cv = I4; x.x_cu = I3 * I4; x.x_cv = 1; x.x_ik = I4;
      } else {
        m.u_src = SRC_P12; g.u_ru = 1; g.u_cu = pb; g.u_k = R14 * R24;
        g.Ru = (int)(R14 * R24); g.K = (int)(R13 * R23);
        m.v_src = SRC_F0 + 2; g.v_rv = 1; g.v_cv = R34; g.v_k = I3 * R34; g.Rv = (int)R34;
        g.Cu = I1 * I2; g.Cv = I3; x.x_cu = I3 * I4; x.x_cv = I4; x.x_ik = 1;
      }
    }
  }
  if (N == 4) {
    const int64_t I1 = I[0], I2 = I[1], I3 = I[2], I4 = I[3];
    const int64_t R12 = R[0][1], R13 = R[0][2], R14 = R[0][3];
    const int64_t R23 = R[1][2], R24 = R[1][3], R34 = R[2][3];
    // P12[(i1,i2)][(r13,r23)][(r14,r24)], contracted over r12, and
    // P34[(i3,i4)][(r13,r14)][(r23,r24)], contracted over r34: the prefix
    // and suffix groups of the general-order chain at N = 4
    if (!chain_desc(factor_layout(P, 0), factor_layout(P, 1), prefix_layout(P, 1), P->es,
                    &P->pgd[0]) ||
        !chain_desc(factor_layout(P, 2), factor_layout(P, 3), suffix_layout(P, 2), P->es,
                    &P->pgd[1]))
      return false;
    P->pnum[0] = I1 * I2 * R13 * R14 * R23 * R24;
    P->pnum[1] = I3 * I4 * R13 * R14 * R23 * R24;
  }
  return true;
}

inline int ld_mod(int x, int r) { return x + ((r - x % 64) % 64 + 64) % 64; }
// Slab row strides for the generator's MFMA operand reads (lane = 16 rows x
// 4 k): [p][kap] rows (lanes read row p0 + l%16 at kap k0 + l/16) need a
// stride that is 4 times an odd number; [kap][p] rows (lanes read row
// k0 + l/16 at p0 + l%16) a stride of 16 mod 32.  Either way the 64 lanes of
// one read hit 64 distinct banks.
inline int ld_pk(int kp) { return kp + ((4 - kp % 8) % 8 + 8) % 8; }
inline int ld_kp(int pp) { return pp + ((16 - pp % 32) % 32 + 32) % 32; }
inline int floor_log2(int x) {
  int l = 0;
  while ((2 << l) <= x) ++l;
  return l;
}

// Operand slabs: [kap][p] (p contiguous; ld = 16 mod 64) unless kap is the
// contiguous index in HBM, then [p][kap] (ld = 4 mod 64).  Both orders give
// bank-conflict-free MFMA operand reads.
void fill_tile(const MGen& mg, int TCu, int TCv, int kalign, TileGeom* tg) {
  tg->TCu = TCu;
  tg->TCv = TCv;
  tg->tcol = TCu * TCv;
  tg->tcolp = (tg->tcol + kalign - 1) / kalign * kalign;
  tg->Pu = mg.Ru * TCu;
  tg->Qv = mg.Rv * TCv;
  tg->Pp = pad16(tg->Pu);
  tg->Qp = pad16(tg->Qv);
  tg->Kp = (mg.K + 3) / 4 * 4;
  if (mg.u_k == 1 && mg.K > 1) {
    tg->us_k = 1; tg->us_p = ld_pk(tg->Kp); tg->u_len = tg->Pp * tg->us_p;
  } else {
    tg->us_p = 1; tg->us_k = ld_kp(tg->Pp); tg->u_len = tg->Kp * tg->us_k;
  }
  if (mg.v_k == 1 && mg.K > 1) {
    tg->vs_k = 1; tg->vs_q = ld_pk(tg->Kp); tg->v_len = tg->Qp * tg->vs_q;
  } else {
    tg->vs_q = 1; tg->vs_k = ld_kp(tg->Qp); tg->v_len = tg->Kp * tg->vs_k;
  }
  // staging lanes along the slab's contiguous index (at most 64)
  tg->u_lw = floor_log2(std::min(tg->us_k == 1 ? tg->Kp : tg->Pp, 64));
  tg->v_lw = floor_log2(std::min(tg->vs_k == 1 ? tg->Kp : tg->Qp, 64));
  // 16-byte staging of [kap][p] slabs: ru contiguous and R a multiple of 4,
  // every other stride a multiple of 4 elements, so that each run of four
  // rows is 16-byte aligned (the operand base pointers are checked at launch)
  auto vec_ok = [&](int64_t f_r, int64_t f_c, int64_t f_k, int R, bool k_fast) {
    return !k_fast && f_r == 1 && R % 4 == 0 && f_c % 4 == 0 && f_k % 4 == 0;
  };
  tg->u_vec = vec_ok(mg.u_ru, mg.u_cu, mg.u_k, mg.Ru, tg->us_k == 1) ? 1 : 0;
  tg->v_vec = vec_ok(mg.v_rv, mg.v_cv, mg.v_k, mg.Rv, tg->vs_k == 1) ? 1 : 0;
  tg->nTileU = (mg.Cu + TCu - 1) / TCu;
  tg->nTileV = (mg.Cv + TCv - 1) / TCv;
  tg->nColTiles = tg->nTileU * tg->nTileV;
}

// Pick the column tile minimizing MFMA instructions (padding included) per
// real column, plus a fixed per-tile overhead, within the LDS budget.
// extra_mfma(tg) is the consumer's work per tile; lds(tg) its LDS bytes.
// rows of the index tables kept in LDS per launch
inline size_t table_bytes(const TileGeom& tg, bool with_cols) {
  return sizeof(SlabRow) * (size_t)(tg.Pp + tg.Qp + (with_cols ? tg.tcolp : 0));
}

template <class Extra, class Lds>
bool choose_tile(const MGen& mg, int mg_repeat, int kalign, Extra extra_mfma, Lds lds,
                 TileGeom* best, size_t lds_shared = 80 * 1024, double mgen_w = 1.0) {
  static const int cv_c[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20, 24, 25, 30, 32, 40, 48, 50, 64};
  static const int cu_c[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  double best_cost = 1e300;
  bool found = false;
  std::vector<int> cvs;
  for (int v : cv_c)
    if (v <= mg.Cv) cvs.push_back(v);
  if (mg.Cv <= 64) cvs.push_back((int)mg.Cv);
  std::vector<int> cus;
  for (int u : cu_c)
    if (u <= mg.Cu) cus.push_back(u);
  if (mg.Cu <= 64) cus.push_back((int)mg.Cu);
  for (int TCv : cvs) {
    for (int TCu : cus) {
      const int tcol = TCu * TCv;
      if (tcol > 256) continue;
      TileGeom tg;
      fill_tile(mg, TCu, TCv, kalign, &tg);
      const size_t bytes = lds(tg);
      if (bytes > (size_t)gram_max_lds_bytes()) continue;
      const double mgen = (double)(tg.Pp / 16) * (tg.Qp / 16) * (tg.Kp / 4) * mg_repeat * mgen_w;
      const double real = ((double)mg.Cu / tg.nTileU) * ((double)mg.Cv / tg.nTileV);
      // staging: the U slab is reloaded when the cu block changes, the V slab
      // when the cv block changes (tiles run cv-block fastest); an element
      // costs about 1/48 of an MFMA instruction
      const double u_per_tile = (double)tg.Kp * tg.Pp / (double)tg.nTileV;
      const double v_per_tile = tg.nTileV > 1 ? (double)tg.Kp * tg.Qp : 0.0;
      const double stage = (u_per_tile + v_per_tile) * mg_repeat / 48.0;
      double cost = (mgen + stage + extra_mfma(tg) + 24.0) / real;
      // above 80 KB only one workgroup fits a CU, and none overlaps its
      // staging with another's MFMA work (measured: 1.3x-1.5x slower)
      if (bytes > lds_shared) cost *= 1.5;
      const double par = (double)tg.nColTiles * mg_repeat;
      if (par < 512.0) cost *= 512.0 / std::max(par, 1.0);   // too few tiles to fill 256 CUs
      // one workgroup per CU: whole tiles per CU, so the last round of the
      // launch is full only if the tile count divides evenly
      if (lds_shared > 80 * 1024 && par >= 256.0)
        cost *= std::ceil(par / 256.0) / (par / 256.0);
      if (cost < best_cost * 0.999) {
        best_cost = cost;
        *best = tg;
        found = true;
      }
    }
  }
  return found;
}

bool setup_geom(ModeInfo& m, size_t es, int prec, bool wide_f32) {
  const bool bf = prec == FCTN_BF16 || prec == FCTN_BF16X3;
  const int nbf = prec == FCTN_BF16X3 ? 2 : 1;   // bf16 copies (hi, lo)
  GramGeom& g = m.geom;
  g.s = (int)m.s;
  g.sp = pad16(g.s);
  g.Ik = (int)m.Ik;
  g.ip = pad16(g.Ik);
  g.nbj = g.sp / 16;
  g.nG = g.nbj * (g.nbj + 1) / 2;
  g.nB = (g.ip / 16) * g.nbj;
  g.nTiles = g.nG + g.nB;
  // float32 modes of 129-448 output tiles with s >= 128: one or two groups
  // of 16 waves x 10, 12 or 14 tiles, so that the sub-network tile is
  // generated and X staged once per column tile for every 160-224 tiles
  // instead of every 128 (video modes 1-2: 75.7/64.9 -> 67.6/59.6 us,
  // multispectral modes 1-2: 56.7/55.4 -> 48.1/47.8 us).  Measured slower:
  // three such groups (new-video modes 1-2, 462 and 498 tiles: 212/180 ->
  // 234/236 us) and s = 96 with 135 tiles, whose single group's X block of
  // all I_k rows cost more than it saved
  const bool wide_groups = prec == FCTN_F32 && g.s >= 128 &&
                           g.nTiles > gram_tiles_per_group() && g.nTiles <= 2 * 16 * 14;
  int tpg = gram_tiles_per_group();
  if (wide_groups) {
    // the fewest groups of at most 16 x 14 tiles, of 16 x 10, 12 or 14
    const int ngr = (g.nTiles + 16 * 14 - 1) / (16 * 14);
    const int per = (g.nTiles + ngr - 1) / ngr;
    const int tpw = std::max(10, ((per + 15) / 16 + 1) / 2 * 2);
    tpg = 16 * tpw;
  }
  g.tilesPerGroup = tpg;
  // Otherwise 16 waves of 8 tiles (one workgroup per CU, all of its LDS) or
  // 8 waves of 16 tiles (two workgroups per CU): 128 tiles per group either
  // way.
  // The bf16 forms take the 16-wave form: their hi/lo tiles need LDS that
  // would leave room for one 8-wave workgroup per CU, and the split form's
  // 16-tile instance needs 243 registers (two waves per SIMD), its 8-tile
  // instance 128 (four); measured on the 144x176x3x50 video shape, modes with
  // s_k = 192: 104/96/158 us -> 73/63/107 us (split), 63/66/109 -> 57/50/86
  // (plain).  float32 takes 16 waves only where the caller asks (modes with
  // a large cached pair or group operand, whose larger column tiles then
  // save restaging: video mode 4 121 -> 105 us, new-video mode 4 881 -> 807,
  // order-5 modes 6-21 % faster) or takes the wider groups above, and keeps
  // two 8-wave workgroups elsewhere (16 waves of 8 tiles cost modes 1-2 of
  // order 4 and the order-3 modes 6-20 %).
  // Modes with at most 16 output tiles run the small-tile instance (8 waves)
  // in every form.
  const bool small_tiles = g.nTiles <= 16;
  g.nw = (prec == FCTN_BF16 || prec == FCTN_BF16X3 || (prec == FCTN_F32 && wide_f32) ||
          wide_groups) &&
                 !small_tiles
             ? 16
             : 8;
  g.nGroups = (g.nTiles + tpg - 1) / tpg;
  int xmax = 0;
  for (int grp = 0; grp < g.nGroups; ++grp) {
    const int t0 = grp * tpg, t1 = std::min(t0 + tpg, g.nTiles);
    if (t1 > g.nG) {
      const int bf = (std::max(t0, g.nG) - g.nG) / g.nbj, bl = (t1 - 1 - g.nG) / g.nbj;
      xmax = std::max(xmax, (bl - bf + 1) * 16);
    }
  }
  g.xrows = xmax;
  // the small-tile kernels give LDS only to the X rows below I_k (and, in
  // float32, to the M rows below s), plus one zero row that the MFMA reads
  // of the padding rows use; their X staging writes the rows below I_k only.
  // Elsewhere every padded row has its own LDS
  g.mrows = g.sp;
  g.xalloc = g.xrows;
  g.zrow = 0;
  if (prec != FCTN_F64 && small_tiles) {
    int xa = 0;
    for (int grp = 0; grp < g.nGroups; ++grp) {
      const int t0 = grp * tpg, t1 = std::min(t0 + tpg, g.nTiles);
      if (t1 > g.nG) {
        const int bf = (std::max(t0, g.nG) - g.nG) / g.nbj, bl = (t1 - 1 - g.nG) / g.nbj;
        xa = std::max(xa, std::min((bl - bf + 1) * 16, g.Ik - bf * 16));
      }
    }
    // the bf16 forms trim the X rows only
    g.mrows = prec == FCTN_F32 ? g.s : g.sp;
    g.xalloc = xa;
    g.zrow = 1;
  }
  // M and X tiles are [row][column]; bf16 rows are tcolp + 8 bf16 values long,
  // float32/float64 rows tcolp + 16 bytes (16-byte aligned after the slabs)
  // bf16 forms with a contraction length of at least 24 generate the
  // sub-network tile in split bf16 from bf16 head/tail slabs ([p][kap], kap
  // padded to a multiple of 32, plus 8)
  const int kp4 = (m.mg.K + 3) / 4 * 4;
  g.mg16 = bf && kp4 >= 24 ? 1 : 0;
  g.ldk = (kp4 + 31) / 32 * 32 + 8;
  auto gram_lds = [&](const TileGeom& tg) {
    if (bf) {
      const size_t slabs = g.mg16 ? (size_t)(tg.Pp + tg.Qp) * g.ldk * 4
                                  : (size_t)(tg.u_len + tg.v_len) * es;
      return slabs + table_bytes(tg, true) +
             ((size_t)(g.sp + g.xalloc) * nbf + g.zrow) * (tg.tcolp + 8) * 2;
    }
    const size_t slabs = (table_bytes(tg, true) + (size_t)(tg.u_len + tg.v_len) * es + 15) &
                         ~(size_t)15;
    return slabs + (size_t)(g.mrows + g.xalloc + g.zrow) * (tg.tcolp + 16 / es) * es;
  };
  // consumer MFMA time per tile in fp32-16x16x4 units (a bf16 16x16x32 issue
  // takes about half as long and covers 8 times the k range)
  auto gram_work = [&](const TileGeom& tg) {
    if (bf) return (double)g.nTiles * (tg.tcolp / 32) * (nbf == 2 ? 3 : 1) * 0.5;
    return (double)g.nTiles * (tg.tcolp / 4);
  };
  // column tiles in whole 16-byte reads per lane group: 4 (16 / es) columns
  // a split-bf16 generator step (three 16x16x32 MFMAs, about half an fp32
  // 16x16x4 issue each) covers 32 kap against the float32 one's 4
  if (!choose_tile(m.mg, g.nGroups, bf ? 32 : 64 / (int)es, gram_work, gram_lds, &g.tg,
                   g.nw == 16 ? (size_t)gram_max_lds_bytes() : (size_t)80 * 1024,
                   g.mg16 ? 1.5 / 8.0 : 1.0))
    return false;
  if (bf) {
    g.ldm = g.tg.tcolp + 8;
  } else {
    g.ldm = g.tg.tcolp + 16 / (int)es;
  }
  g.ldx = g.ldm;
  g.lds_bytes = gram_lds(g.tg);
  int64_t ns = std::max<int64_t>(1, (g.nw == 16 ? 256 : kTargetGramWGs) / g.nGroups);
  // a multiple of the XCD count, so that rounding the split count up below
  // keeps the launch within one round of the CUs
  if (ns >= kXcds) ns = ns / kXcds * kXcds;
  ns = std::min<int64_t>(ns, g.tg.nColTiles);
  g.colTilesPerSplit = (g.tg.nColTiles + ns - 1) / ns;
  g.nSplit = (int32_t)((g.tg.nColTiles + g.colTilesPerSplit - 1) / g.colTilesPerSplit);
  // a whole number of splits per XCD (the trailing ones may hold no column
  // tile: they write zero partial sums), so that the kernel can give each
  // XCD a contiguous range of them
  if (g.nSplit >= kXcds) g.nSplit = (g.nSplit + kXcds - 1) / kXcds * kXcds;

  RecGeom& r = m.rg;
  r.s = g.s;
  r.sp = g.sp;
  r.Ik = g.Ik;
  r.ip = g.ip;
  // rows of the staged A_k(k) and of the M tile 16 bytes apart modulo 256:
  // the 16 lanes of one 16-byte read hit distinct banks
  const int lda = ld_mod(r.sp, 4);
  // A_k(k) in LDS only when small: a large copy would leave room for one
  // workgroup per CU (it is read through the cache otherwise)
  const bool stage_a = (size_t)r.ip * lda * es <= 24 * 1024;
  r.lda = stage_a ? lda : 0;
  auto rec_lds = [&](const TileGeom& tg) {
    const int ldm = ld_mod(std::max(r.sp, 4), 4);
    return (size_t)(tg.u_len + tg.v_len + (size_t)pad16(tg.tcolp) * ldm + (size_t)r.ip * r.lda) *
               es + table_bytes(tg, false) + 16;
  };
  auto rec_work = [&](const TileGeom& tg) {
    return (double)(r.ip / 16) * (pad16(tg.tcolp) / 16) * (r.sp / 4);
  };
  if (!choose_tile(m.mg, 1, 4, rec_work, rec_lds, &r.tg)) return false;
  r.tg.tcolp = pad16(r.tg.tcol);
  r.ldm = ld_mod(std::max(r.sp, 4), 4);
  r.lds_bytes = rec_lds(r.tg);
  // two workgroups per CU, each walking a contiguous range of column tiles
  r.nblk = (int32_t)std::min<int64_t>(r.tg.nColTiles, 512);
  return r.lds_bytes <= (size_t)gram_max_lds_bytes();
}

// carve (or measure, base == nullptr) the workspace; returns bytes
size_t carve(fctn_plan_s* P, char* base) {
  Carver c{base, 0};
  const int N = P->N;
  const size_t es = P->es;
  const size_t acc_es = P->prec == FCTN_F64 ? 8 : 4;
  P->X = c.take(P->numel * es);
  P->Z = c.take(P->numel * es);
  P->bits = (uint32_t*)c.take(((P->numel + 63) / 64) * 2 * sizeof(uint32_t));
  P->bad_nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (P->numel + 255) / 256));
  P->bad_part = (int32_t*)c.take(P->bad_nblk * sizeof(int32_t));
  P->bad_flag = (int32_t*)c.take(sizeof(int32_t));
  P->dev_err = (int32_t*)c.take(sizeof(int32_t));
  int64_t smax = 1, imax = 1;
  P->max_cls = 1;
  size_t part_bytes = 0;
  for (int k = 0; k < N; ++k) {
    const ModeInfo& m = P->mode[k];
    P->A64[k] = (double*)c.take(P->fnum[k] * sizeof(double));
    P->Aw[k] = c.take(P->fnum[k] * es);
    P->Au[k] = c.take(P->fnum[k] * es);
    P->Q[k] = (double*)c.take(m.Ik * m.Ik * sizeof(double));
    P->Qt[k] = (double*)c.take(m.Ik * m.Ik * sizeof(double));
    P->lamcol[k] = (double*)c.take(m.Ik * sizeof(double));
    smax = std::max(smax, m.s);
    imax = std::max(imax, m.Ik);
    P->max_cls = std::max(P->max_cls, m.ncls);
    part_bytes = std::max(part_bytes, (size_t)m.geom.nSplit * m.geom.nTiles * 256 * acc_es);
  }
  for (int p = 0; p < 2; ++p) P->P[p] = (N == 4) ? c.take(P->pnum[p] * es) : nullptr;
  for (int q = 0; q < P->ngrp; ++q) P->grp[q].buf = c.take(P->grp[q].num * es);
  P->part = c.take(part_bytes);
  P->part_cur = P->part;
  P->part_bytes = part_bytes;
  P->G = (double*)c.take(smax * smax * sizeof(double));
  P->B = (double*)c.take(imax * smax * sizeof(double));
  P->At = (double*)c.take(imax * smax * sizeof(double));
  P->trace_part = (double*)c.take((size_t)N * P->max_cls * sizeof(double));
  P->lam_half = (double*)c.take(N * sizeof(double));
  P->ncls_dev = (int32_t*)c.take(N * sizeof(int32_t));
  P->xblocks = x_update_blocks(P->prec, P->numel);
  P->xpart = (double*)c.take((size_t)P->xblocks * 3 * sizeof(double));
  P->hist = (double*)c.take(kHist * 4 * sizeof(double));
  P->scratch_slot = (double*)c.take(4 * sizeof(double));
  return align256(c.off);
}

bool init_plan_struct(const fctn_desc* d, fctn_plan_s* P) {
  memset(P, 0, sizeof(*P));
  P->d = *d;
  P->N = d->order;
  P->prec = d->precision;
  P->es = P->prec == FCTN_F64 ? 8 : 4;
  P->numel = 1;
  for (int k = 0; k < P->N; ++k) {
    P->dims[k] = d->dims[k];
    P->numel *= d->dims[k];
  }
  fill_ranks(d, P->R);
  for (int k = 0; k < P->N; ++k) {
    int64_t n = 1;
    for (int j = 0; j < P->N; ++j) n *= (j == k) ? P->dims[k] : P->R[k][j];
    P->fnum[k] = n;
  }
  if (!setup_modes(P)) return false;
  // the kernels index X, the factors and the pair tensors with 32-bit offsets
  if (P->numel >= ((int64_t)1 << 31)) return false;
  for (int p = 0; p < 2; ++p)
    if (P->pnum[p] >= ((int64_t)1 << 31)) return false;
  for (int k = 0; k < P->N; ++k)
    if (P->fnum[k] >= ((int64_t)1 << 31)) return false;
  for (int k = 0; k < P->N; ++k) {
    if (!solve_supported((int32_t)P->mode[k].s)) return false;
    // float32 Gram of the modes whose large operand is a cached pair or
    // group (modes 3-4 of order 4, every mode of orders >= 5): one 16-wave
    // workgroup per CU, whose LDS budget lets the column tiles grow
    if (!setup_geom(P->mode[k], P->es, P->prec, P->N >= 5 || (P->N == 4 && k >= 2)))
      return false;
  }
  const char* gp = getenv("FCTN_GEOM");
  if (gp && gp[0] == '1') {
    for (int k = 0; k < P->N; ++k) {
      const GramGeom& g = P->mode[k].geom;
      const RecGeom& r = P->mode[k].rg;
      fprintf(stderr,
              "mode %d: s %d Ik %d | gram tile %dx%d (P %d/%d Q %d/%d K %d; slabs %s %s) "
              "cols %lld groups %d splits %d waves %d lds %zu | rec tile %dx%d lds %zu "
              "stageA %d blocks %d\n",
              k, g.s, g.Ik, g.tg.TCu, g.tg.TCv, g.tg.Pu, g.tg.Pp, g.tg.Qv, g.tg.Qp, g.tg.Kp,
              g.tg.us_k == 1 ? "[p][k]" : "[k][p]", g.tg.vs_k == 1 ? "[q][k]" : "[k][q]",
              (long long)g.tg.nColTiles, g.nGroups, g.nSplit, g.nw, g.lds_bytes, r.tg.TCu,
              r.tg.TCv, r.lds_bytes, r.lda > 0, r.nblk);
    }
  }
  return true;
}

const void* src_ptr(fctn_plan_s* P, int src) {
  if (src == SRC_P12) return P->P[0];
  if (src == SRC_P34) return P->P[1];
  if (src >= SRC_GRP) return P->grp[src - SRC_GRP].buf;
  return P->Aw[src - SRC_F0];
}

#define FCTN_LAUNCH(P, expr)                                  \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ == hipSuccess && (P)->debug) e_ = hipStreamSynchronize((P)->st); \
    if (e_ != hipSuccess) {                                   \
      (P)->sticky = FCTN_E_DEVICE;                            \
      return FCTN_E_DEVICE;                                   \
    }                                                         \
  } while (0)

hipEvent_t prof_event(fctn_plan_s* P) {
  hipEvent_t e = nullptr;
  if (!P->prof->pool.empty()) {
    e = P->prof->pool.back();
    P->prof->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// event pair around one launch when profiling is on
#define FCTN_TIMED(P, stage, flops, bytes, expr)                         \
  do {                                                                   \
    hipEvent_t a_ = nullptr, b_ = nullptr;                               \
    if ((P)->prof_on) {                                                  \
      a_ = prof_event(P);                                                \
      b_ = prof_event(P);                                                \
      if (a_) hipEventRecord(a_, (P)->st);                               \
    }                                                                    \
    FCTN_LAUNCH(P, expr);                                                \
    if (a_ && b_) {                                                      \
      hipEventRecord(b_, (P)->st);                                       \
      (P)->prof->recs.push_back(ProfRec{(stage), a_, b_, (double)(flops), (double)(bytes)}); \
    }                                                                    \
  } while (0)

// pair p is built from factors (0,1) for p = 0 and (2,3) for p = 1
fctn_status ensure_pair(fctn_plan_s* P, int p, bool force) {
  const int fa = p == 0 ? 0 : 2, fb = fa + 1;
  if (!force && P->pvalid[p] && P->pver[p][0] == P->fver[fa] && P->pver[p][1] == P->fver[fb])
    return FCTN_OK;
  GroupDesc gd = P->pgd[p];
  gd.F[0] = P->Aw[fa];
  gd.F[1] = P->Aw[fb];
  FCTN_TIMED(P, FCTN_STAGE_PAIR, 2.0 * P->pnum[p] * gd.inner,
             (double)(P->fnum[fa] + P->fnum[fb] + P->pnum[p]) * P->es,
             launch_group(P->prec, gd, P->P[p], P->st));
  P->pvalid[p] = true;
  P->pver[p][0] = P->fver[fa];
  P->pver[p][1] = P->fver[fb];
  return FCTN_OK;
}

int pair_of_mode(int N, int k) {
  if (N != 4) return -1;
  return (k <= 1) ? 1 : 0;
}

// orders N >= 5: (re)build group q (and first, where needed, the group it
// grows from) unless it was built from the current versions of its factors;
// with force (Algorithm 1) every call rebuilds the chain from the factors
fctn_status ensure_group(fctn_plan_s* P, int q, bool force) {
  GroupSlot& G = P->grp[q];
  bool fresh = G.built && !force;
  for (int f = 0; f < P->N && fresh; ++f)
    if (((G.fmask >> f) & 1u) && G.snap[f] != P->fver[f]) fresh = false;
  if (fresh) return FCTN_OK;
  GroupDesc gd = G.gd;
  for (int a = 0; a < 2; ++a) {
    if (G.src[a] >= SRC_GRP) {
      fctn_status s = ensure_group(P, G.src[a] - SRC_GRP, force);
      if (s != FCTN_OK) return s;
    }
    gd.F[a] = src_ptr(P, G.src[a]);
  }
  FCTN_TIMED(P, FCTN_STAGE_PAIR, 2.0 * gd.total * gd.inner,
             (double)gd.total * P->es, launch_group(P->prec, gd, G.buf, P->st));
  G.built = true;
  for (int f = 0; f < P->N; ++f) G.snap[f] = P->fver[f];
  return FCTN_OK;
}

fctn_status ensure_groups(fctn_plan_s* P, int k) {
  const ModeInfo& m = P->mode[k];
  for (int src : {m.u_src, m.v_src})
    if (src >= SRC_GRP) {
      fctn_status s = ensure_group(P, src - SRC_GRP, P->d.reuse == 0);
      if (s != FCTN_OK) return s;
    }
  return FCTN_OK;
}

fctn_status prepare_mode(fctn_plan_s* P, int k) {
  if (P->N >= 5) return ensure_groups(P, k);
  const int p = pair_of_mode(P->N, k);
  if (p >= 0) return ensure_pair(P, p, P->d.reuse == 0);
  return FCTN_OK;
}

MGen resolved_mgen(fctn_plan_s* P, int k) {
  MGen g = P->mode[k].mg;
  g.U = src_ptr(P, P->mode[k].u_src);
  g.V = src_ptr(P, P->mode[k].v_src);
  return g;
}

fctn_status gram_rhs(fctn_plan_s* P, int k, double* G, double* B) {
  fctn_status s = prepare_mode(P, k);
  if (s != FCTN_OK) return s;
  const ModeInfo& m = P->mode[k];
  const MGen g = resolved_mgen(P, k);
  const double sC = (double)m.s * m.C;
  const double acc_es = P->prec == FCTN_F64 ? 8.0 : 4.0;
  const double part_bytes = (double)m.geom.nSplit * m.geom.nTiles * 256 * acc_es;
  FCTN_TIMED(P, FCTN_STAGE_GRAM_RHS, 2.0 * sC * (m.mg.K + m.s + m.Ik),
             (double)P->numel * P->es + part_bytes,
             launch_gram_rhs(P->prec, g, P->X, m.xv, m.geom, P->part_cur, P->st));
  FCTN_TIMED(P, FCTN_STAGE_REDUCE, (double)m.geom.nSplit * (m.s * m.s + m.Ik * m.s),
             part_bytes + 8.0 * (m.s * m.s + 2 * m.Ik * m.s),
             launch_reduce_gb(P->prec, m.geom, P->part_cur, P->A64[k], m.spost, P->d.rho, G, B,
                              P->st));
  return FCTN_OK;
}

fctn_status solve(fctn_plan_s* P, int k, const double* G, const double* B) {
  const ModeInfo& m = P->mode[k];
  const double s3 = (double)m.s * m.s * m.s;
  const double tr_flops = 2.0 * m.Ik * m.Ik * m.s;
  const double tr_bytes = 8.0 * (m.Ik * m.Ik + 2.0 * m.Ik * m.s);
  // b~ = Q^T B into At; the solves overwrite each class's rows with a~
  FCTN_TIMED(P, FCTN_STAGE_TRANSFORM, tr_flops, tr_bytes,
             launch_project(P->Qt[k], B, (int32_t)m.Ik, (int32_t)m.s, P->At, P->st));
  FCTN_TIMED(P, FCTN_STAGE_SOLVE, m.ncls * (s3 / 3.0 + 4.0 * m.s * m.s),
             8.0 * (m.s * m.s + 2.0 * m.Ik * m.s),
             launch_solve_classes(G, (int32_t)m.Ik, (int32_t)m.s, P->d.lambda[k],
                                  P->d.delta[k], P->d.rho, P->At,
                                  P->trace_part + (size_t)k * P->max_cls, P->dev_err, P->st));
  // with the asymmetric extrapolation the epilogue also reads the proximal
  // centre A_k^t (overwritten in place), and the trace term the solve wrote
  // for the un-extrapolated factor is recomputed for the new one
  const bool ext = P->d.extrap_alpha > 0.0;
  FCTN_TIMED(P, FCTN_STAGE_TRANSFORM, tr_flops + (ext ? 3.0 * m.Ik * m.s : 0.0),
             tr_bytes + 2.0 * m.Ik * m.s * P->es + (ext ? 8.0 * m.Ik * m.s : 0.0),
             launch_backtransform(P->prec, P->Q[k], P->At, (int32_t)m.Ik, (int32_t)m.s,
                                  m.spost, P->d.extrap_alpha, P->d.extrap_beta, P->A64[k],
                                  P->Aw[k], P->Au[k], P->st));
  if (ext)
    FCTN_TIMED(P, FCTN_STAGE_TRANSFORM, 4.0 * m.Ik * m.s, 8.0 * m.Ik * m.s,
               launch_factor_trace(P->A64[k], (int32_t)m.Ik, (int32_t)m.s, m.spost,
                                   P->d.delta[k], (int32_t)m.ncls,
                                   P->trace_part + (size_t)k * P->max_cls, P->st));
  P->fver[k]++;
  return FCTN_OK;
}

fctn_status reconstruct(fctn_plan_s* P, int k, void* Z) {
  const int p = pair_of_mode(P->N, k);
  if (p >= 0) {
    fctn_status s = ensure_pair(P, p, P->d.reuse == 0);
    if (s != FCTN_OK) return s;
  }
  if (P->N >= 5) {
    fctn_status s = ensure_groups(P, k);
    if (s != FCTN_OK) return s;
  }
  const ModeInfo& m = P->mode[k];
  const MGen g = resolved_mgen(P, k);
  FCTN_TIMED(P, FCTN_STAGE_RECONSTRUCT, 2.0 * (double)m.s * m.C * (m.mg.K + m.Ik),
             (double)P->numel * P->es,
             launch_reconstruct(P->prec, g, P->Au[k], Z, m.xv, m.rg, P->st));
  return FCTN_OK;
}

fctn_status x_update(fctn_plan_s* P, const void* Z, double* slot, bool with_trace) {
  FCTN_TIMED(P, FCTN_STAGE_XUPDATE, 5.0 * P->numel,
             3.0 * P->numel * P->es + P->numel / 8.0,
             launch_x_update(P->prec, P->X, Z, P->bits, P->d.rho, P->numel, P->xblocks, P->xpart,
                             P->st));
  FCTN_TIMED(P, FCTN_STAGE_STATS, 3.0 * P->xblocks, 24.0 * P->xblocks,
             launch_stats(P->xpart, P->xblocks, P->trace_part, P->lam_half, P->ncls_dev,
                          with_trace ? P->N : 0, P->max_cls, slot, P->st));
  return FCTN_OK;
}

void sweep_order(const fctn_plan_s* P, int64_t t, int* order) {
  for (int k = 0; k < P->N; ++k) order[k] = k;
  if (P->d.order_policy == 1 && P->N == 4 && (t % 2) == 1) {
    order[0] = 2; order[1] = 3; order[2] = 0; order[3] = 1;
  }
}

// host-side ranges for rocprofv3 --marker-trace: one per sweep and one per
// factor block inside it (no cost without a profiler attached)
struct Range {
  explicit Range(const char* m) { roctxRangePushA(m); }
  ~Range() { roctxRangePop(); }
};
const char* const kModeRange[FCTN_MAX_ORDER] = {"fctn factor 1", "fctn factor 2", "fctn factor 3",
                                                "fctn factor 4", "fctn factor 5", "fctn factor 6",
                                                "fctn factor 7", "fctn factor 8"};

fctn_status one_sweep(fctn_plan_s* P) {
  Range sweep_range("fctn sweep");
  int order[FCTN_MAX_ORDER];
  sweep_order(P, P->sweeps_done, order);
  fctn_status s;
  for (int n = 0; n < P->N; ++n) {
    const int k = order[n];
    Range mode_range(kModeRange[k]);
    if ((s = gram_rhs(P, k, P->G, P->B)) != FCTN_OK) return s;
    if ((s = solve(P, k, P->G, P->B)) != FCTN_OK) return s;
  }
  const int last = order[P->N - 1];
  {
    Range x_range("fctn X step");
    if ((s = reconstruct(P, last, P->Z)) != FCTN_OK) return s;
    if ((s = x_update(P, P->Z, P->hist + (P->sweeps_done % kHist) * 4, true)) != FCTN_OK)
      return s;
  }
  P->sweeps_done++;
  return FCTN_OK;
}

// Synchronizes the plan's stream and reports a kernel-side failure (the
// device error word) as FCTN_E_DEVICE, sticky.
fctn_status sync_checked(fctn_plan_s* P) {
  int32_t err = 0;
  if (hipMemcpyAsync(&err, P->dev_err, sizeof(err), hipMemcpyDeviceToHost, P->st) !=
          hipSuccess ||
      hipStreamSynchronize(P->st) != hipSuccess || err != 0) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return FCTN_OK;
}

// Standard normal draws for the initial factors from a seed (Algorithm 1's
// initialization).  Counter-based: value i of the stream depends only on
// (seed, i).  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) gives 64-bit
// words w_j = mix(seed + (j + 1) * 0x9E3779B97F4A7C15); pair n of normals
// comes from words 2n and 2n + 1 by the Box-Muller transform (u1 in (0, 1]
// and u2 in [0, 1) from the top 53 bits): r = sqrt(-2 ln u1), values
// r cos(2 pi u2) and r sin(2 pi u2).  Factor 1's entries take stream
// indices 0 .. |A_1| - 1, factor 2's the next ones, and so on.
uint64_t splitmix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double seeded_normal(uint64_t seed, uint64_t i) {
  const uint64_t n = i / 2;
  const double u1 = ((double)(splitmix64(seed, 2 * n) >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(splitmix64(seed, 2 * n + 1) >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double a = 6.283185307179586 * u2;
  return (i & 1) ? r * sin(a) : r * cos(a);
}

fctn_status read_slot(fctn_plan_s* P, const double* slot, fctn_sweep_stats* out) {
  double h[4];
  if (hipMemcpyAsync(h, slot, sizeof(h), hipMemcpyDeviceToHost, P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  fctn_status v = sync_checked(P);
  if (v != FCTN_OK) return v;
  out->rel_change = h[0];
  out->f_data = h[1];
  out->f_trace = h[2];
  out->objective = h[3];
  for (int i = 0; i < 8; ++i) out->ms_stage[i] = 0.f;
  return FCTN_OK;
}

// ms_stage of the sweeps whose launches were recorded from record `from` on
// (per-kernel timing on; the stream is synchronized)
void stage_times(fctn_plan_s* P, size_t from, int nsweeps, fctn_sweep_stats* out) {
  if (!P->prof || nsweeps <= 0) return;
  double ms[8] = {};
  for (size_t i = from; i < P->prof->recs.size(); ++i) {
    float t = 0.f;
    const ProfRec& r = P->prof->recs[i];
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) ms[r.stage] += t;
  }
  for (int i = 0; i < 8; ++i) out->ms_stage[i] = (float)(ms[i] / nsweeps);
}

// Plan set-up without host synchronization or pageable copies, so that it
// can be queued on a stream that other plans are using.
fctn_status plan_build(const fctn_desc* desc, void* ws_dev, size_t ws_bytes, hipStream_t st,
                       fctn_plan_s** out) {
  *out = nullptr;
  fctn_status v = validate(desc);
  if (v != FCTN_OK) return v;
  if (!ws_dev || ((uintptr_t)ws_dev & 255)) return FCTN_E_INVALID;
  fctn_plan_s* P = new (std::nothrow) fctn_plan_s;
  if (!P) return FCTN_E_NOMEM;
  if (!init_plan_struct(desc, P)) {
    delete P;
    return FCTN_E_UNSUPPORTED;
  }
  const size_t need = carve(P, nullptr);
  if (ws_bytes < need) {
    delete P;
    return FCTN_E_NOMEM;
  }
  carve(P, (char*)ws_dev);
  P->st = st;
  const char* dbg = getenv("FCTN_DEBUG");
  P->debug = dbg && dbg[0] == '1';
  // zero state, bases, per-mode constants
  bool ok = hipMemsetAsync(ws_dev, 0, need, P->st) == hipSuccess;
  PlanConsts pc{};
  pc.n = P->N;
  for (int k = 0; k < P->N && ok; ++k) {
    ok = launch_build_basis(P->Q[k], P->Qt[k], P->lamcol[k], (int32_t)P->mode[k].Ik,
                            desc->delta[k], P->st) == hipSuccess;
    pc.lam_half[k] = 0.5 * desc->lambda[k];
    pc.ncls[k] = P->mode[k].ncls;
  }
  ok = ok && launch_set_consts(P->lam_half, P->ncls_dev, pc, P->st) == hipSuccess;
  if (!ok) {
    delete P;
    return FCTN_E_DEVICE;
  }
  *out = P;
  return FCTN_OK;
}

// float64 factors from device memory (concatenated in mode order), then the
// working-precision copies; asynchronous on the plan's stream
fctn_status set_factors_dev(fctn_plan_s* P, const double* A_dev) {
  int64_t off = 0;
  for (int k = 0; k < P->N; ++k) {
    if (hipMemcpyAsync(P->A64[k], A_dev + off, P->fnum[k] * sizeof(double),
                       hipMemcpyDeviceToDevice, P->st) != hipSuccess) {
      P->sticky = FCTN_E_DEVICE;
      return FCTN_E_DEVICE;
    }
    off += P->fnum[k];
    const ModeInfo& m = P->mode[k];
    FCTN_LAUNCH(P, launch_cast_factor(P->prec, P->A64[k], P->Aw[k], P->Au[k], (int32_t)m.Ik,
                                      (int32_t)m.s, m.spost, P->st));
    P->fver[k]++;
  }
  P->pvalid[0] = P->pvalid[1] = false;
  return FCTN_OK;
}

// X = P_Omega(Y), the mask bits and the non-finite flag (P->bad_flag[0]);
// asynchronous on the plan's stream
fctn_status set_observed_async(fctn_plan_s* P, const void* Y_dev, const uint8_t* mask_dev) {
  FCTN_LAUNCH(P, launch_init_observed(P->prec, Y_dev, mask_dev, P->X, P->bits, P->bad_part,
                                      P->numel, P->bad_nblk, P->st));
  FCTN_LAUNCH(P, launch_any_flag(P->bad_part, P->bad_nblk, P->bad_flag, P->st));
  return FCTN_OK;
}

}  // namespace

extern "C" {

size_t fctn_workspace_bytes(const fctn_desc* desc) {
  if (validate(desc) != FCTN_OK) return 0;
  fctn_plan_s* P = new (std::nothrow) fctn_plan_s;
  if (!P) return 0;
  size_t bytes = 0;
  if (init_plan_struct(desc, P)) bytes = carve(P, nullptr);
  delete P;
  return bytes;
}

fctn_status fctn_mode_sizes(const fctn_desc* desc, int32_t k, int64_t* s_k, int64_t* I_k) {
  fctn_status v = validate(desc);
  if (v != FCTN_OK) return v;
  if (k < 0 || k >= desc->order || !s_k || !I_k) return FCTN_E_INVALID;
  int R[FCTN_MAX_ORDER][FCTN_MAX_ORDER];
  fill_ranks(desc, R);
  int64_t s = 1;
  for (int j = 0; j < desc->order; ++j)
    if (j != k) s *= R[k][j];
  *s_k = s;
  *I_k = desc->dims[k];
  return FCTN_OK;
}

fctn_status fctn_plan(const fctn_desc* desc, void* ws_dev, size_t ws_bytes, void* hip_stream,
                      const double* const* A0_host, uint64_t seed, fctn_plan_t* out) {
  if (!out) return FCTN_E_INVALID;
  *out = nullptr;
  fctn_plan_s* P = nullptr;
  fctn_status v = plan_build(desc, ws_dev, ws_bytes, (hipStream_t)hip_stream, &P);
  if (v != FCTN_OK) return v;
  if (hipStreamSynchronize(P->st) != hipSuccess) {
    delete P;
    return FCTN_E_DEVICE;
  }
  // initial factors: the caller's, or standard normal draws from the seed
  std::vector<std::vector<double>> drawn;
  std::vector<const double*> ptrs(P->N);
  if (A0_host) {
    for (int k = 0; k < P->N; ++k) ptrs[k] = A0_host[k];
  } else {
    uint64_t i = 0;
    drawn.resize(P->N);
    for (int k = 0; k < P->N; ++k) {
      drawn[k].resize(P->fnum[k]);
      for (int64_t e = 0; e < P->fnum[k]; ++e) drawn[k][e] = seeded_normal(seed, i++);
      ptrs[k] = drawn[k].data();
    }
  }
  v = fctn_set_factors(P, ptrs.data());
  if (v != FCTN_OK) {
    delete P;
    return v;
  }
  *out = P;
  return FCTN_OK;
}

fctn_status fctn_set_factors(fctn_plan_t P, const double* const* A_host) {
  if (!P || !A_host) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  for (int k = 0; k < P->N; ++k)
    if (!A_host[k]) return FCTN_E_INVALID;
  for (int k = 0; k < P->N; ++k) {
    if (hipMemcpyAsync(P->A64[k], A_host[k], P->fnum[k] * sizeof(double), hipMemcpyHostToDevice,
                       P->st) != hipSuccess) {
      P->sticky = FCTN_E_DEVICE;
      return FCTN_E_DEVICE;
    }
    const ModeInfo& m = P->mode[k];
    FCTN_LAUNCH(P, launch_cast_factor(P->prec, P->A64[k], P->Aw[k], P->Au[k], (int32_t)m.Ik,
                                      (int32_t)m.s, m.spost, P->st));
    P->fver[k]++;
  }
  if (hipStreamSynchronize(P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  P->pvalid[0] = P->pvalid[1] = false;
  return FCTN_OK;
}

fctn_status fctn_set_observed(fctn_plan_t P, const void* Y_dev, const uint8_t* mask_dev) {
  if (!P || !Y_dev || !mask_dev) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  fctn_status v = set_observed_async(P, Y_dev, mask_dev);
  if (v != FCTN_OK) return v;
  int32_t bad = 0;
  if (hipMemcpyAsync(&bad, P->bad_flag, sizeof(bad), hipMemcpyDeviceToHost, P->st) !=
          hipSuccess ||
      hipStreamSynchronize(P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return bad ? FCTN_E_NUMERIC : FCTN_OK;
}

fctn_status fctn_set_factors_dev(fctn_plan_t P, const double* A_dev) {
  if (!P || !A_dev) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  return set_factors_dev(P, A_dev);
}

fctn_status fctn_set_x(fctn_plan_t P, const void* X_dev) {
  if (!P || !X_dev) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  if (hipMemcpyAsync(P->X, X_dev, P->numel * P->es, hipMemcpyDeviceToDevice, P->st) !=
      hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return FCTN_OK;
}

fctn_status fctn_get_sweep_index(fctn_plan_t P, int64_t* t_host) {
  if (!P || !t_host) return FCTN_E_INVALID;
  *t_host = P->sweeps_done;
  return FCTN_OK;
}

fctn_status fctn_set_sweep_index(fctn_plan_t P, int64_t t) {
  if (!P || t < 0) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  P->sweeps_done = t;
  P->hist_first = t;
  return FCTN_OK;
}

fctn_status fctn_regrow(fctn_plan_t to, fctn_plan_t from, const double* fill_dev) {
  if (!to || !from || !fill_dev || to == from) return FCTN_E_INVALID;
  if (to->sticky != FCTN_OK) return to->sticky;
  if (from->sticky != FCTN_OK) return from->sticky;
  if (to->N != from->N || to->prec != from->prec) return FCTN_E_INVALID;
  const int N = to->N;
  for (int k = 0; k < N; ++k)
    if (to->dims[k] != from->dims[k]) return FCTN_E_INVALID;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (i != j && to->R[i][j] < from->R[i][j]) return FCTN_E_INVALID;
  // from's pending work (its X and factors) before to's stream reads them
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, from->st) != hipSuccess || hipStreamWaitEvent(to->st, ev, 0) != hipSuccess) {
    if (ev) hipEventDestroy(ev);
    to->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  bool ok = hipMemcpyAsync(to->X, from->X, to->numel * to->es, hipMemcpyDeviceToDevice,
                           to->st) == hipSuccess &&
            hipMemcpyAsync(to->bits, from->bits, ((to->numel + 63) / 64) * 2 * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, to->st) == hipSuccess;
  int64_t off = 0;
  for (int k = 0; k < N && ok; ++k) {
    RegrowDesc d{};
    d.N = N;
    for (int j = 0; j < N; ++j) {
      d.shape_old[j] = j == k ? from->dims[k] : from->R[k][j];
      d.shape_new[j] = j == k ? to->dims[k] : to->R[k][j];
      if (j < k) d.zero_modes |= 1u << j;
    }
    ok = launch_regrow(from->A64[k], fill_dev + off, to->A64[k], d, to->st) == hipSuccess;
    const ModeInfo& m = to->mode[k];
    ok = ok && launch_cast_factor(to->prec, to->A64[k], to->Aw[k], to->Au[k], (int32_t)m.Ik,
                                  (int32_t)m.s, m.spost, to->st) == hipSuccess;
    to->fver[k]++;
    off += to->fnum[k];
  }
  to->pvalid[0] = to->pvalid[1] = false;
  ok = ok && hipStreamSynchronize(to->st) == hipSuccess;
  hipEventDestroy(ev);
  if (!ok) {
    to->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return FCTN_OK;
}

fctn_status fctn_sweep(fctn_plan_t P, int32_t nsweeps, fctn_sweep_stats* stats_host) {
  if (!P || nsweeps < 0) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  size_t last_from = 0;
  for (int32_t i = 0; i < nsweeps; ++i) {
    if (P->prof) last_from = P->prof->recs.size();
    fctn_status s = one_sweep(P);
    if (s != FCTN_OK) return s;
  }
  if (stats_host) {
    if (P->sweeps_done == P->hist_first) {
      memset(stats_host, 0, sizeof(*stats_host));
      return FCTN_OK;
    }
    fctn_status s = read_slot(P, P->hist + ((P->sweeps_done - 1) % kHist) * 4, stats_host);
    if (s == FCTN_OK && P->prof_on && nsweeps > 0) stage_times(P, last_from, 1, stats_host);
    return s;
  }
  return FCTN_OK;
}

}  // extern "C"

namespace {

// The split-K partial products of fctn_sweep_noalloc live in this array
// instead of the plan's workspace.  In host code `scratch` only names the
// symbol: its device address, one per device, comes from
// hipGetSymbolAddress and is what kernels receive.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of `st` (looked up once per
// device, with that device current; the caller's current device is restored).
fctn_status static_scratch(hipStream_t st, void** out) {
  int dev = 0;
  if (hipStreamGetDevice(st, &dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return FCTN_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return FCTN_E_DEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return FCTN_E_DEVICE;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return FCTN_E_DEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FCTN_OK;
}

}  // namespace

extern "C" {

fctn_status fctn_sweep_noalloc(fctn_plan_t P, int32_t nsweeps) {
  if (!P || nsweeps < 0) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  if (P->part_bytes > kStaticScratchBytes) return FCTN_E_NOMEM;
  void* ptr = nullptr;
  fctn_status v = static_scratch(P->st, &ptr);
  if (v != FCTN_OK) return v;
  // every partial tile is written by the Gram pass before the reduction reads
  // it, so nothing in the array needs clearing
  // per-kernel timing records events into growing host lists: off here
  const bool prof = P->prof_on;
  P->prof_on = false;
  P->part_cur = ptr;
  for (int32_t i = 0; i < nsweeps && v == FCTN_OK; ++i) v = one_sweep(P);
  P->part_cur = P->part;
  P->prof_on = prof;
  return v;
}

fctn_status fctn_sweep_many(fctn_plan_t* plans, int32_t count, int32_t nsweeps) {
  if (!plans || count < 0 || nsweeps < 0) return FCTN_E_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    if (!plans[i]) return FCTN_E_INVALID;
    if (plans[i]->sticky != FCTN_OK) return plans[i]->sticky;
  }
  // round-robin one sweep per plan so that work queued on distinct streams overlaps
  for (int32_t t = 0; t < nsweeps; ++t)
    for (int32_t i = 0; i < count; ++i) {
      fctn_status s = one_sweep(plans[i]);
      if (s != FCTN_OK) return s;
    }
  return FCTN_OK;
}

fctn_status fctn_complete(fctn_plan_t P, int32_t max_sweeps, double tol, int32_t check_every,
                          void* X_out_dev, fctn_stats* stats_host) {
  if (!P || max_sweeps < 0 || check_every < 1) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  int32_t done = 0;
  fctn_sweep_stats last{};
  bool have_last = false;
  while (done < max_sweeps) {
    const int32_t n = std::min(check_every, max_sweeps - done);
    for (int32_t i = 0; i < n; ++i) {
      fctn_status s = one_sweep(P);
      if (s != FCTN_OK) return s;
    }
    done += n;
    if (tol > 0.0) {
      fctn_status s = read_slot(P, P->hist + ((P->sweeps_done - 1) % kHist) * 4, &last);
      if (s != FCTN_OK) return s;
      have_last = true;
      if (last.rel_change <= tol) break;
    }
  }
  if (X_out_dev) {
    if (hipMemcpyAsync(X_out_dev, P->X, P->numel * P->es, hipMemcpyDeviceToDevice, P->st) !=
        hipSuccess) {
      P->sticky = FCTN_E_DEVICE;
      return FCTN_E_DEVICE;
    }
  }
  if (stats_host) {
    stats_host->sweeps_done = done;
    if (done > 0 && !have_last) {
      fctn_status s = read_slot(P, P->hist + ((P->sweeps_done - 1) % kHist) * 4, &last);
      if (s != FCTN_OK) return s;
    } else if (X_out_dev) {
      // the X_out copy was queued after the last stopping-rule read: a caller
      // that asked for host stats gets a finished X_out as well
      fctn_status s = sync_checked(P);
      if (s != FCTN_OK) return s;
    }
    stats_host->rel_change = done > 0 ? last.rel_change : 0.0;
    stats_host->objective = done > 0 ? last.objective : 0.0;
  }
  return FCTN_OK;
}

fctn_status fctn_get_history(fctn_plan_t P, int32_t first, int32_t count,
                             fctn_sweep_stats* out_host) {
  if (!P || !out_host || first < 0 || count < 0) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  if ((int64_t)first + count > P->sweeps_done || P->sweeps_done - first > kHist ||
      first < P->hist_first)
    return FCTN_E_INVALID;
  std::vector<double> h((size_t)kHist * 4);
  if (hipMemcpyAsync(h.data(), P->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                     P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  fctn_status v = sync_checked(P);
  if (v != FCTN_OK) return v;
  for (int32_t i = 0; i < count; ++i) {
    const double* e = &h[((first + i) % kHist) * 4];
    out_host[i].rel_change = e[0];
    out_host[i].f_data = e[1];
    out_host[i].f_trace = e[2];
    out_host[i].objective = e[3];
    for (int k = 0; k < 8; ++k) out_host[i].ms_stage[k] = 0.f;
  }
  return FCTN_OK;
}

fctn_status fctn_get_x(fctn_plan_t P, void* dst_dev) {
  if (!P || !dst_dev) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  if (hipMemcpyAsync(dst_dev, P->X, P->numel * P->es, hipMemcpyDeviceToDevice, P->st) !=
      hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return FCTN_OK;
}

fctn_status fctn_get_factor(fctn_plan_t P, int32_t k, double* dst_dev) {
  if (!P || !dst_dev || k < 0 || k >= P->N) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  if (hipMemcpyAsync(dst_dev, P->A64[k], P->fnum[k] * sizeof(double), hipMemcpyDeviceToDevice,
                     P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  return FCTN_OK;
}

fctn_status fctn_step_gram_rhs(fctn_plan_t P, int32_t k, double* G_dev, double* B_dev) {
  if (!P || !G_dev || !B_dev || k < 0 || k >= P->N) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  return gram_rhs(P, k, G_dev, B_dev);
}

fctn_status fctn_step_solve(fctn_plan_t P, int32_t k, const double* G_dev, const double* B_dev,
                            double* trace_host) {
  if (!P || !G_dev || !B_dev || k < 0 || k >= P->N) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  fctn_status s = solve(P, k, G_dev, B_dev);
  if (s != FCTN_OK) return s;
  if (trace_host) {
    const int nc = P->mode[k].ncls;
    std::vector<double> tp(nc);
    if (hipMemcpyAsync(tp.data(), P->trace_part + (size_t)k * P->max_cls, nc * sizeof(double),
                       hipMemcpyDeviceToHost, P->st) != hipSuccess) {
      P->sticky = FCTN_E_DEVICE;
      return FCTN_E_DEVICE;
    }
    fctn_status v = sync_checked(P);
    if (v != FCTN_OK) return v;
    double t = 0.0;
    for (double v : tp) t += v;
    *trace_host = t;
  }
  return FCTN_OK;
}

fctn_status fctn_step_reconstruct(fctn_plan_t P, int32_t k, void* Z_dev) {
  if (!P || !Z_dev || k < 0 || k >= P->N) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  return reconstruct(P, k, Z_dev);
}

fctn_status fctn_step_x_update(fctn_plan_t P, const void* Z_dev, fctn_sweep_stats* stats_host) {
  if (!P || !Z_dev || ((uintptr_t)Z_dev & 15)) return FCTN_E_INVALID;
  if (P->sticky != FCTN_OK) return P->sticky;
  // the trace term is not part of this step's scalars
  fctn_status s = x_update(P, Z_dev, P->scratch_slot, false);
  if (s != FCTN_OK) return s;
  if (stats_host) return read_slot(P, P->scratch_slot, stats_host);
  return FCTN_OK;
}

fctn_status fctn_profile_enable(fctn_plan_t P, int32_t enable) {
  if (!P) return FCTN_E_INVALID;
  if (enable && !P->prof) {
    P->prof = new (std::nothrow) ProfState;
    if (!P->prof) return FCTN_E_NOMEM;
  }
  P->prof_on = enable != 0;
  return FCTN_OK;
}

fctn_status fctn_profile_read(fctn_plan_t P, fctn_profile* out, int32_t reset) {
  if (!P || !out) return FCTN_E_INVALID;
  memset(out, 0, sizeof(*out));
  if (!P->prof) return FCTN_OK;
  if (hipStreamSynchronize(P->st) != hipSuccess) {
    P->sticky = FCTN_E_DEVICE;
    return FCTN_E_DEVICE;
  }
  for (const ProfRec& r : P->prof->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return FCTN_E_DEVICE;
    out->launches[r.stage] += 1;
    out->ms[r.stage] += ms;
    out->flops[r.stage] += r.flops;
    out->bytes[r.stage] += r.bytes;
  }
  if (reset) {
    for (const ProfRec& r : P->prof->recs) {
      P->prof->pool.push_back(r.a);
      P->prof->pool.push_back(r.b);
    }
    P->prof->recs.clear();
  }
  return FCTN_OK;
}

fctn_status fctn_destroy(fctn_plan_t P) {
  if (!P) return FCTN_E_INVALID;
  hipStreamSynchronize(P->st);
  if (P->prof) {
    for (const ProfRec& r : P->prof->recs) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    for (hipEvent_t e : P->prof->pool) hipEventDestroy(e);
    delete P->prof;
  }
  delete P;
  return FCTN_OK;
}

const char* fctn_status_str(fctn_status s) {
  switch (s) {
    case FCTN_OK: return "ok";
    case FCTN_E_INVALID: return "invalid argument";
    case FCTN_E_NOMEM: return "workspace too small";
    case FCTN_E_DEVICE: return "HIP runtime error";
    case FCTN_E_NUMERIC: return "non-finite observed value";
    case FCTN_E_UNSUPPORTED: return "unsupported configuration";
    case FCTN_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Continuous batching: independent completions share one GPU.  Each admitted
// request is a plan carved from the server's arena; its sweeps are queued on
// one of the caller's streams, at most `depth` at a time, one sweep per
// request per round so that requests sharing a stream interleave.  Requests
// are admitted first-in first-out as slots and arena room free up.
// ---------------------------------------------------------------------------
namespace {

double mono_now() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct SrvPending {
  fctn_request r;
  size_t bytes;
  double t_submit;
};

struct SrvSlot {
  bool busy = false;
  bool finishing = false;
  bool cancelled = false;
  fctn_plan_s* plan = nullptr;
  size_t off = 0, bytes = 0;
  int32_t enq = 0;
  std::deque<hipEvent_t> inflight;
  hipEvent_t done = nullptr;
  fctn_request req{};
  double t_submit = 0.0, t_admit = 0.0;
};

}  // namespace

struct fctn_server_s {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes; disjoint, coalesced
  size_t used = 0;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  int depth = 1;
  std::vector<SrvSlot> slots;
  std::deque<SrvPending> queue;
  std::deque<fctn_completion> dropped;   // cancelled before admission
  std::vector<hipEvent_t> pool;
  int32_t* pin_flag = nullptr;  // pinned host memory, two flags per slot: the
                                // non-finite flag of Y and the device error word
  double* pin_stats = nullptr;  // pinned host memory, four doubles per slot
  fctn_status sticky = FCTN_OK;
};

namespace {

bool arena_alloc(fctn_server_s* S, size_t bytes, size_t* off) {
  for (auto it = S->free_.begin(); it != S->free_.end(); ++it) {
    if (it->second < bytes) continue;
    *off = it->first;
    const size_t rest = it->second - bytes;
    S->free_.erase(it);
    if (rest > 0) S->free_[*off + bytes] = rest;
    S->used += bytes;
    return true;
  }
  return false;
}

void arena_free(fctn_server_s* S, size_t off, size_t bytes) {
  S->used -= bytes;
  auto it = S->free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != S->free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    S->free_.erase(nx);
  }
  if (it != S->free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      S->free_.erase(it);
    }
  }
}

hipEvent_t srv_event(fctn_server_s* S) {
  if (!S->pool.empty()) {
    hipEvent_t e = S->pool.back();
    S->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

fctn_status srv_fail(fctn_server_s* S, fctn_status v) {
  S->sticky = v;
  return v;
}

// set-up of an admitted request on stream st (no host synchronization)
fctn_status srv_admit(fctn_server_s* S, int slot, const SrvPending& h, size_t off,
                      hipStream_t st) {
  fctn_plan_s* P = nullptr;
  fctn_status v = plan_build(&h.r.desc, S->arena + off, h.bytes, st, &P);
  if (v != FCTN_OK) return v;
  v = set_factors_dev(P, h.r.A0_dev);
  if (v == FCTN_OK) v = set_observed_async(P, h.r.Y_dev, h.r.mask_dev);
  if (v == FCTN_OK && hipMemcpyAsync(S->pin_flag + 2 * slot, P->bad_flag, sizeof(int32_t),
                                     hipMemcpyDeviceToHost, st) != hipSuccess)
    v = FCTN_E_DEVICE;
  if (v != FCTN_OK) {
    delete P;
    return v;
  }
  SrvSlot& sl = S->slots[slot];
  sl.busy = true;
  sl.finishing = false;
  sl.plan = P;
  sl.off = off;
  sl.bytes = h.bytes;
  sl.enq = 0;
  sl.req = h.r;
  sl.t_submit = h.t_submit;
  sl.t_admit = mono_now();
  return FCTN_OK;
}

// results of a request whose sweeps are all queued: X out, last-sweep
// scalars to pinned memory, then the completion event
fctn_status srv_finish(fctn_server_s* S, int slot) {
  SrvSlot& sl = S->slots[slot];
  fctn_plan_s* P = sl.plan;
  if (hipMemcpyAsync(sl.req.X_out_dev, P->X, P->numel * P->es, hipMemcpyDeviceToDevice,
                     P->st) != hipSuccess)
    return FCTN_E_DEVICE;
  if (hipMemcpyAsync(S->pin_flag + 2 * slot + 1, P->dev_err, sizeof(int32_t),
                     hipMemcpyDeviceToHost, P->st) != hipSuccess)
    return FCTN_E_DEVICE;
  double* ps = S->pin_stats + 4 * slot;
  if (P->sweeps_done > 0) {
    if (hipMemcpyAsync(ps, P->hist + ((P->sweeps_done - 1) % kHist) * 4, 4 * sizeof(double),
                       hipMemcpyDeviceToHost, P->st) != hipSuccess)
      return FCTN_E_DEVICE;
  } else {
    ps[0] = ps[1] = ps[2] = ps[3] = 0.0;
  }
  sl.done = srv_event(S);
  if (!sl.done || hipEventRecord(sl.done, P->st) != hipSuccess) return FCTN_E_DEVICE;
  sl.finishing = true;
  return FCTN_OK;
}

}  // namespace

extern "C" {

fctn_status fctn_server_create(void* arena_dev, size_t arena_bytes, void* const* streams,
                               int32_t nstreams, int32_t max_active, int32_t depth,
                               fctn_server_t* out) {
  if (!out) return FCTN_E_INVALID;
  *out = nullptr;
  if (!arena_dev || ((uintptr_t)arena_dev & 255) || arena_bytes < 256 || !streams ||
      nstreams < 1 || max_active < 1 || depth < 1)
    return FCTN_E_INVALID;
  fctn_server_s* S = new (std::nothrow) fctn_server_s;
  if (!S) return FCTN_E_NOMEM;
  S->arena = (char*)arena_dev;
  S->arena_bytes = arena_bytes & ~(size_t)255;
  S->free_[0] = S->arena_bytes;
  for (int i = 0; i < nstreams; ++i) S->streams.push_back((hipStream_t)streams[i]);
  S->depth = depth;
  S->slots.resize(max_active);
  if (hipHostMalloc((void**)&S->pin_flag, sizeof(int32_t) * 2 * max_active, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&S->pin_stats, sizeof(double) * 4 * max_active,
                    hipHostMallocDefault) != hipSuccess) {
    if (S->pin_flag) hipHostFree(S->pin_flag);
    delete S;
    return FCTN_E_DEVICE;
  }
  *out = S;
  return FCTN_OK;
}

fctn_status fctn_server_submit(fctn_server_t S, const fctn_request* r) {
  if (!S || !r) return FCTN_E_INVALID;
  if (S->sticky != FCTN_OK) return S->sticky;
  fctn_status v = validate(&r->desc);
  if (v != FCTN_OK) return v;
  if (!r->Y_dev || !r->mask_dev || !r->A0_dev || !r->X_out_dev || r->sweeps < 0)
    return FCTN_E_INVALID;
  const size_t bytes = align256(fctn_workspace_bytes(&r->desc));
  if (bytes == 0) return FCTN_E_UNSUPPORTED;
  if (bytes > S->arena_bytes) return FCTN_E_NOMEM;
  S->queue.push_back(SrvPending{*r, bytes, mono_now()});
  return FCTN_OK;
}

fctn_status fctn_server_step(fctn_server_t S, fctn_completion* done, int32_t max_done,
                             int32_t* n_done) {
  if (!S || !n_done || max_done < 0 || (max_done > 0 && !done)) return FCTN_E_INVALID;
  *n_done = 0;
  if (S->sticky != FCTN_OK) return S->sticky;
  const int ns = (int)S->slots.size();
  // requests cancelled while queued
  while (!S->dropped.empty() && *n_done < max_done) {
    done[(*n_done)++] = S->dropped.front();
    S->dropped.pop_front();
  }
  // retire
  for (int i = 0; i < ns && *n_done < max_done; ++i) {
    SrvSlot& sl = S->slots[i];
    if (!sl.busy || !sl.finishing) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return srv_fail(S, FCTN_E_DEVICE);
    fctn_completion& c = done[(*n_done)++];
    c.tag = sl.req.tag;
    c.status = S->pin_flag[2 * i + 1] ? FCTN_E_DEVICE
               : sl.cancelled          ? FCTN_E_CANCELLED
               : S->pin_flag[2 * i]    ? FCTN_E_NUMERIC
                                       : FCTN_OK;
    c.sweeps_done = sl.enq;
    c.rel_change = S->pin_stats[4 * i + 0];
    c.objective = S->pin_stats[4 * i + 3];
    c.t_submit = sl.t_submit;
    c.t_admit = sl.t_admit;
    c.t_done = mono_now();
    S->pool.push_back(sl.done);
    sl.done = nullptr;
    for (hipEvent_t e : sl.inflight) S->pool.push_back(e);
    sl.inflight.clear();
    delete sl.plan;
    sl.plan = nullptr;
    arena_free(S, sl.off, sl.bytes);
    sl.busy = sl.finishing = sl.cancelled = false;
  }
  // admit, first in first out: the head of the queue waits for room
  while (!S->queue.empty()) {
    int slot = -1;
    for (int i = 0; i < ns; ++i)
      if (!S->slots[i].busy) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    const SrvPending& h = S->queue.front();
    size_t off = 0;
    if (!arena_alloc(S, h.bytes, &off)) break;
    hipStream_t st = S->streams[S->next_stream];
    S->next_stream = (S->next_stream + 1) % (int)S->streams.size();
    fctn_status v = srv_admit(S, slot, h, off, st);
    if (v != FCTN_OK) {
      arena_free(S, off, h.bytes);
      return srv_fail(S, v);
    }
    S->queue.pop_front();
  }
  // progress: rounds of one sweep per request until every request has
  // `depth` sweeps in flight or all of its sweeps queued
  for (bool more = true; more;) {
    more = false;
    for (int i = 0; i < ns; ++i) {
      SrvSlot& sl = S->slots[i];
      if (!sl.busy || sl.finishing) continue;
      while (!sl.inflight.empty()) {
        const hipError_t q = hipEventQuery(sl.inflight.front());
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return srv_fail(S, FCTN_E_DEVICE);
        S->pool.push_back(sl.inflight.front());
        sl.inflight.pop_front();
      }
      if ((int)sl.inflight.size() < S->depth && sl.enq < sl.req.sweeps) {
        fctn_status v = one_sweep(sl.plan);
        if (v != FCTN_OK) return srv_fail(S, v);
        hipEvent_t e = srv_event(S);
        if (!e || hipEventRecord(e, sl.plan->st) != hipSuccess)
          return srv_fail(S, FCTN_E_DEVICE);
        sl.inflight.push_back(e);
        sl.enq++;
        more = true;
      }
      if (sl.enq == sl.req.sweeps) {
        fctn_status v = srv_finish(S, i);
        if (v != FCTN_OK) return srv_fail(S, v);
      }
    }
  }
  return FCTN_OK;
}

fctn_status fctn_server_cancel(fctn_server_t S, uint64_t tag) {
  if (!S) return FCTN_E_INVALID;
  if (S->sticky != FCTN_OK) return S->sticky;
  for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
    if (it->r.tag != tag) continue;
    fctn_completion c{};
    c.tag = tag;
    c.status = FCTN_E_CANCELLED;
    c.t_submit = it->t_submit;
    c.t_done = mono_now();
    S->dropped.push_back(c);
    S->queue.erase(it);
    return FCTN_OK;
  }
  for (SrvSlot& sl : S->slots) {
    if (!sl.busy || sl.finishing || sl.cancelled || sl.req.tag != tag) continue;
    // no further sweeps: fctn_server_step finishes it once the queued ones
    // have run (or at once if none was queued yet)
    sl.cancelled = true;
    sl.req.sweeps = sl.enq;
    return FCTN_OK;
  }
  return FCTN_E_INVALID;
}

fctn_status fctn_server_query(fctn_server_t S, int32_t* queued, int32_t* active,
                              size_t* arena_used) {
  if (!S) return FCTN_E_INVALID;
  if (queued) *queued = (int32_t)S->queue.size();
  if (active) {
    int32_t a = 0;
    for (const SrvSlot& sl : S->slots) a += sl.busy ? 1 : 0;
    *active = a;
  }
  if (arena_used) *arena_used = S->used;
  return S->sticky;
}

fctn_status fctn_server_destroy(fctn_server_t S) {
  if (!S) return FCTN_E_INVALID;
  for (hipStream_t st : S->streams) hipStreamSynchronize(st);
  for (SrvSlot& sl : S->slots) {
    for (hipEvent_t e : sl.inflight) hipEventDestroy(e);
    if (sl.done) hipEventDestroy(sl.done);
    delete sl.plan;
  }
  for (hipEvent_t e : S->pool) hipEventDestroy(e);
  hipHostFree(S->pin_flag);
  hipHostFree(S->pin_stats);
  delete S;
  return FCTN_OK;
}

}  // extern "C"
