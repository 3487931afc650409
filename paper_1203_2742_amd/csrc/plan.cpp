// Symbolic analysis on the host: elimination tree, filled-pattern test,
// supernodes and clique tree (Pothen-Sun), relative indices, level
// schedules and canonical flop counts.
//
// Sections 2 (elimination trees, eqs. e-filled, e-etree-ch), 6.1 (cliques,
// representative vertices, eq. e-repr-test), 6.2 (supernode partitions,
// eq. e-new2), 6.3 (clique trees) and Algorithm 6.1 of the paper.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "mfb_internal.h"

namespace mfb {

static mfb_status_t validate(int64_t n, const int64_t* cp, const int32_t* ri) {
  if (n < 0 || !cp) return MFB_EINVAL;
  if (n > 0 && !ri) return MFB_EINVAL;
  if (n >= (int64_t(1) << 31)) return MFB_EINVAL;
  if (cp[0] != 0) return MFB_EINVAL;
  for (int64_t j = 0; j < n; ++j) {
    if (cp[j + 1] <= cp[j]) return MFB_EINVAL;
    if (ri[cp[j]] != j) return MFB_EINVAL;  // diagonal first
    for (int64_t p = cp[j] + 1; p < cp[j + 1]; ++p)
      if (ri[p] <= ri[p - 1] || ri[p] >= n) return MFB_EINVAL;
  }
  return MFB_OK;
}

static mfb_status_t finish_plan(int64_t n, const int64_t* cp, const int32_t* ri, uint32_t flags,
                                const PlanTuning& tune, const std::vector<std::vector<int32_t>>& members,
                                const std::vector<int32_t>& spar0, mfb_plan_s* p);

mfb_status_t build_plan(int64_t n, const int64_t* cp, const int32_t* ri, uint32_t flags, mfb_plan_s* p,
                        const PlanTuning& tune) {
  mfb_status_t st = validate(n, cp, ri);
  if (st) return st;

  // Elimination tree: parent(j) = min I_j (the first off-diagonal row).
  std::vector<int32_t> epar(n), deg(n);
  for (int64_t j = 0; j < n; ++j) {
    deg[j] = int32_t(cp[j + 1] - cp[j] - 1);
    epar[j] = deg[j] > 0 ? ri[cp[j] + 1] : -1;
  }
  // Filled test: I_j \ {parent} must lie inside I_parent (eq. e-etree-ch);
  // applied to every column this is equivalent to eq. e-filled.
  for (int64_t j = 0; j < n; ++j) {
    if (epar[j] < 0) continue;
    int64_t q = cp[epar[j]] + 1, qe = cp[epar[j] + 1];
    for (int64_t t = cp[j] + 2; t < cp[j + 1]; ++t) {
      while (q < qe && ri[q] < ri[t]) ++q;
      if (q == qe || ri[q] != ri[t]) return MFB_ENOTCHORDAL;
      ++q;
    }
  }
  // Children lists of the elimination tree, ascending.
  std::vector<int32_t> ehead(n, -1), enext(n, -1);
  for (int64_t j = n - 1; j >= 0; --j)
    if (epar[j] >= 0) { enext[j] = ehead[epar[j]]; ehead[epar[j]] = int32_t(j); }

  // Algorithm 6.1 (Pothen-Sun): vertex i is representative iff
  // |I_i| > |I_j| - 1 for every child j (eq. e-repr-test); otherwise it joins
  // the supernode of an eligible child (|I_i| = |I_j| - 1).  The choice among
  // eligible children is free; we take the lowest (or highest) label.
  const bool tie_last = (flags & MFB_PLAN_TIE_LAST) != 0;
  std::vector<int32_t> sn_of(n, -1);
  std::vector<std::vector<int32_t>> members;
  for (int64_t i = 0; i < n; ++i) {
    int32_t pick = -1;
    for (int32_t j = ehead[i]; j != -1; j = enext[j]) {
      if (deg[i] == deg[j] - 1) {
        if (pick < 0 || tie_last) pick = j;
        if (!tie_last) break;
      }
    }
    if (pick < 0) {
      sn_of[i] = int32_t(members.size());
      members.push_back({int32_t(i)});
    } else {
      sn_of[i] = sn_of[pick];
      members[sn_of[i]].push_back(int32_t(i));
    }
  }
  const int32_t ns = int32_t(members.size());
  // Clique-tree parent: the supernode holding the first ancestor
  // min A_s = parent of the last vertex of N_s (Section 6.2).
  std::vector<int32_t> spar0(ns, -1);
  for (int32_t s = 0; s < ns; ++s) {
    int32_t last = members[s].back();
    if (epar[last] >= 0) spar0[s] = sn_of[epar[last]];
  }
  return finish_plan(n, cp, ri, flags, tune, members, spar0, p);
}

// The plan of a supernode partition (members ascending, clique-tree parent
// spar0) of a pattern: clique-tree postorder, the supernode property of
// every column (column c of a supernode holds rows J_s[c:]), relative
// indices, schedules and counts.
static mfb_status_t finish_plan(int64_t n, const int64_t* cp, const int32_t* ri, uint32_t flags,
                                const PlanTuning& tune, const std::vector<std::vector<int32_t>>& members,
                                const std::vector<int32_t>& spar0, mfb_plan_s* p) {
  p->n = n;
  p->nnz = n ? cp[n] : 0;
  p->flags = flags;
  const int32_t ns = int32_t(members.size());
  // Postorder of the clique tree; children visited in order of their
  // representative vertex, roots likewise.
  std::vector<int32_t> chead(ns, -1), cnext(ns, -1);
  for (int32_t s = ns - 1; s >= 0; --s)
    if (spar0[s] >= 0) { cnext[s] = chead[spar0[s]]; chead[spar0[s]] = s; }
  std::vector<int32_t> post;  // post[k] = old id
  post.reserve(ns);
  {
    std::vector<int32_t> stack;
    std::vector<int32_t> it(ns, -2);
    for (int32_t r = 0; r < ns; ++r) {
      if (spar0[r] >= 0) continue;
      stack.push_back(r);
      while (!stack.empty()) {
        int32_t s = stack.back();
        if (it[s] == -2) it[s] = chead[s];
        int32_t c = it[s];
        if (c != -1) {
          it[s] = cnext[c];
          stack.push_back(c);
        } else {
          post.push_back(s);
          stack.pop_back();
        }
      }
    }
  }
  if (int32_t(post.size()) != ns) return MFB_EINVAL;
  std::vector<int32_t> newid(ns);
  for (int32_t k = 0; k < ns; ++k) newid[post[k]] = k;

  p->ns = ns;
  p->N.resize(ns);
  p->J.resize(ns);
  p->parent.resize(ns);
  p->rep.resize(ns);
  p->colbase.resize(ns + 1);
  p->relbase.resize(ns + 1);
  p->arena.resize(ns + 1);
  p->snode_of.resize(n);
  p->col.resize(n);
  p->vlabel.resize(n);
  int64_t cb = 0, rb = 0, ab = 0;
  p->max_front = p->max_ncols = p->max_nanc = 0;
  for (int32_t k = 0; k < ns; ++k) {
    const auto& mem = members[post[k]];
    const int32_t rep = mem[0];
    const int32_t Nn = int32_t(mem.size());
    const int32_t Jn = int32_t(cp[rep + 1] - cp[rep]);
    const int32_t An = Jn - Nn;
    if (An < 0) return MFB_ENOTCHORDAL;
    p->N[k] = Nn;
    p->J[k] = Jn;
    p->rep[k] = rep;
    p->parent[k] = spar0[post[k]] >= 0 ? newid[spar0[post[k]]] : -1;
    p->colbase[k] = int32_t(cb);
    p->relbase[k] = int32_t(rb);
    p->arena[k] = ab;
    // Column c of the supernode holds rows J_s[c:] (eq. e-new2): check.
    const int32_t* Js = ri + cp[rep];
    for (int32_t c = 0; c < Nn; ++c) {
      const int32_t v = mem[c];
      if (Js[c] != v) return MFB_ENOTCHORDAL;
      if (cp[v + 1] - cp[v] != Jn - c) return MFB_ENOTCHORDAL;
      if (std::memcmp(ri + cp[v], Js + c, sizeof(int32_t) * size_t(Jn - c)) != 0)
        return MFB_ENOTCHORDAL;
      p->col[cb + c] = cp[v];
      p->vlabel[cb + c] = v;
      p->snode_of[v] = k;
    }
    cb += Nn;
    rb += An;
    ab += int64_t(An) * (An + 1) / 2;
    p->max_front = std::max(p->max_front, Jn);
    p->max_ncols = std::max(p->max_ncols, Nn);
    p->max_nanc = std::max(p->max_nanc, An);
  }
  p->colbase[ns] = int32_t(cb);
  p->relbase[ns] = int32_t(rb);
  p->arena[ns] = ab;
  p->update_doubles = ab;

  // Relative indices: position of A_s[t] in J_parent(s).  A_s lies inside
  // J_parent (first clique-tree property, Section 6.3).
  p->rel.resize(rb);
  for (int32_t k = 0; k < ns; ++k) {
    const int32_t An = p->J[k] - p->N[k];
    if (An == 0) {
      if (p->parent[k] >= 0) return MFB_ENOTCHORDAL;
      continue;
    }
    if (p->parent[k] < 0) return MFB_ENOTCHORDAL;
    const int32_t* As = ri + cp[p->rep[k]] + p->N[k];
    const int32_t pr = p->rep[p->parent[k]];
    const int32_t* Jp = ri + cp[pr];
    const int32_t Jpn = p->J[p->parent[k]];
    int32_t q = 0;
    for (int32_t t = 0; t < An; ++t) {
      while (q < Jpn && Jp[q] < As[t]) ++q;
      if (q == Jpn || Jp[q] != As[t]) return MFB_ENOTCHORDAL;
      p->rel[p->relbase[k] + t] = q++;
    }
  }
  // Children in postorder numbering (ascending = fixed assembly order).
  p->cptr.assign(ns + 1, 0);
  for (int32_t k = 0; k < ns; ++k)
    if (p->parent[k] >= 0) p->cptr[p->parent[k] + 1]++;
  for (int32_t k = 0; k < ns; ++k) p->cptr[k + 1] += p->cptr[k];
  p->cidx.assign(std::max(1, p->cptr[ns]), 0);
  {
    std::vector<int32_t> fill(p->cptr.begin(), p->cptr.end() - 1);
    for (int32_t k = 0; k < ns; ++k)
      if (p->parent[k] >= 0) p->cidx[fill[p->parent[k]]++] = k;
  }
  // Level schedules.  Height: leaves 0, parent = 1 + max child (postorder
  // visits children first).  Depth: roots 0.
  std::vector<int32_t> h(ns, 0), d(ns, 0);
  int32_t H = 0, Dm = 0;
  for (int32_t k = 0; k < ns; ++k)
    if (p->parent[k] >= 0) h[p->parent[k]] = std::max(h[p->parent[k]], h[k] + 1);
  for (int32_t k = ns - 1; k >= 0; --k)
    if (p->parent[k] >= 0) d[k] = d[p->parent[k]] + 1;
  for (int32_t k = 0; k < ns; ++k) { H = std::max(H, h[k]); Dm = std::max(Dm, d[k]); }
  auto make_levels = [&](const std::vector<int32_t>& lv, int32_t nl, std::vector<int32_t>& list,
                         std::vector<Level>& levels) {
    levels.assign(ns ? nl + 1 : 0, Level{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    list.clear();
    list.reserve(ns);
    std::vector<int32_t> cnt(nl + 2, 0);
    for (int32_t k = 0; k < ns; ++k) cnt[lv[k] + 1]++;
    for (int32_t l = 0; l <= nl; ++l) cnt[l + 1] += cnt[l];
    list.assign(ns, 0);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t k = 0; k < ns; ++k) list[fill[lv[k]]++] = k;
    for (int32_t l = 0; ns && l <= nl; ++l) {
      Level L{cnt[l], cnt[l + 1] - cnt[l], 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t t = L.begin; t < L.begin + L.count; ++t) {
        int32_t k = list[t];
        L.maxN = std::max(L.maxN, p->N[k]);
        L.maxA = std::max(L.maxA, p->J[k] - p->N[k]);
        L.maxJ = std::max(L.maxJ, p->J[k]);
        const double Nn = p->N[k], Jn = p->J[k], An = Jn - Nn;
        L.p += Nn * Jn - Nn * (Nn - 1) / 2;
        L.u += An * (An + 1) / 2;
        L.n3 += Nn * Nn * Nn;
        L.n2a += Nn * Nn * An;
        L.na2 += Nn * An * An;
        L.a3 += An * An * An;
      }
      levels[l] = L;
    }
  };
  make_levels(h, H, p->up_list, p->up_levels);
  make_levels(d, Dm, p->down_list, p->down_levels);

  // Class-split copies of the schedules (see ClassSeg).  A register
  // kernel of class c takes any front of order <= kRegMax[c], so all the
  // register fronts of a level go into one launch at the largest class
  // they need: small fronts then run beside the large ones instead of in
  // launches of their own after them.
  //
  // The Hessian down-sweep register kernels stage their operands in chunks
  // and step through A (or J) columns one at a time, with most of the
  // register front idle when N is small: they beat the blocked kernels on
  // levels of small fronts (every J <= kDownRegMaxJ) and on levels of roots
  // (every A = 0), and lose elsewhere; the projected inverse follows the
  // same rule.
  //
  // Wide fronts (J above the wide threshold, N <= kWideMaxN, A > 0) of the
  // level-scheduled sweeps go to a segment of their own (cls == kWide),
  // launched first on their level, with their tiles numbered: 64 x 64 lower
  // tiles of the A x A block and 64-row tiles of the A rows.
  p->wide_thr = (flags & MFB_PLAN_WIDE_LOW) ? kWideJLow : kWideJ;
  // (never below kVExplicitMax: the tile-parallel path leaves C_V^-1, the
  // representation of the larger blocks)
  p->big_a = (flags & MFB_PLAN_WIDE_LOW) ? kVExplicitMax : kBigA;
  // the two thresholds (front order above which fronts run tile-parallel;
  // ancestor count above which S_AA is factored tile-parallel): the plan
  // options when given, else the environment overrides, else the defaults
  if (!(flags & MFB_PLAN_WIDE_LOW)) {
    if (const char* e = std::getenv("MFB_WIDE_J")) p->wide_thr = std::max(kWideJLow, std::atoi(e));
    if (const char* e = std::getenv("MFB_BIG_A")) p->big_a = std::max(kVExplicitMax, std::atoi(e));
  }
  if (tune.wide_j > 0) p->wide_thr = tune.wide_j;
  if (tune.big_a > 0) p->big_a = tune.big_a;
  // every front above the threshold is wide in the root-to-leaf sweeps; in
  // the leaf-to-root ones those with at most kWideMaxN columns (and an
  // update block) are wide and the others fat
  auto is_wide = [&](int32_t k) { return p->J[k] > p->wide_thr; };
  auto up_class = [&](int32_t k) {
    if (!is_wide(k)) return -1;
    return p->N[k] > kWideMaxN ? kFat : (p->J[k] > p->N[k] ? kWide : -1);
  };
  auto number_tiles = [&](ClassSched& cs, ClassSeg& g) {
    auto tl = [](int32_t m) { return (m + kWideTile - 1) / kWideTile; };
    const Level& S = g.lv;
    int32_t acc = 0;
    g.aa_off = int32_t(cs.pre.size());
    for (int32_t t = S.begin; t < S.begin + S.count; ++t) {
      cs.pre.push_back(acc);
      const int32_t na = tl(p->J[cs.list[t]] - p->N[cs.list[t]]);
      acc += na * (na + 1) / 2;
    }
    cs.pre.push_back(acc);
    g.n_aa = acc;
    g.an_off = int32_t(cs.pre.size());
    acc = 0;
    for (int32_t t = S.begin; t < S.begin + S.count; ++t) {
      cs.pre.push_back(acc);
      acc += tl(p->J[cs.list[t]] - p->N[cs.list[t]]) * tl(p->N[cs.list[t]]);
    }
    cs.pre.push_back(acc);
    g.n_an = acc;
    g.nn_off = int32_t(cs.pre.size());
    acc = 0;
    for (int32_t t = S.begin; t < S.begin + S.count; ++t) {
      cs.pre.push_back(acc);
      acc += tl(p->N[cs.list[t]]) * tl(p->N[cs.list[t]]);
    }
    cs.pre.push_back(acc);
    g.n_nn = acc;
    g.fat_panel = g.fat_fin = 0;
    for (int32_t t = S.begin; t < S.begin + S.count; ++t) {
      const int32_t k = cs.list[t], tn = tl(p->N[k]), ta = tl(p->J[k] - p->N[k]);
      g.fat_panel = std::max(g.fat_panel, tl(p->J[k]) * tn);
      g.fat_fin = std::max(g.fat_fin, tn * tn + ta * tn);
    }
  };
  // mid_wide: the Hessian's root-to-leaf sweep also takes the non-root
  // fronts above kDownRegMaxJ tile-parallel (wide class)
  bool mid_wide = false;
  auto down_wide = [&](int32_t k) {
    return is_wide(k) || (mid_wide && p->J[k] > kDownRegMaxJ && p->J[k] != p->N[k]);
  };
  auto down_reg_level = [&](const std::vector<int32_t>& list, const Level& L, bool wide_ok) {
    bool small = true, roots = true;
    for (int32_t t = L.begin; t < L.begin + L.count; ++t) {
      if (wide_ok && down_wide(list[t])) continue;
      small = small && p->J[list[t]] <= kDownRegMaxJ;
      roots = roots && p->J[list[t]] == p->N[list[t]];
    }
    return small || roots;
  };
  auto make_classes = [&](const std::vector<int32_t>& list, const std::vector<Level>& levels,
                          bool by_a, bool down, ClassSched& cs, bool wide_ok) {
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    cs.list.reserve(ns);
    auto fit_class = [&](int32_t k) {  // smallest class that holds the front, or kRegClasses
      const int32_t m = by_a ? p->J[k] - p->N[k] : p->J[k];
      int c = 0;
      while (c < kRegClasses && m > kRegMax[c]) ++c;
      return c;
    };
    for (int32_t l = 0; l < int32_t(levels.size()); ++l) {
      const Level& L = levels[l];
      const bool reg_ok = !down || down_reg_level(list, L, wide_ok);
      int lvcls = 0;
      for (int32_t t = L.begin; t < L.begin + L.count; ++t)
        if (!(wide_ok && (down ? down_wide(list[t]) : is_wide(list[t]))) && fit_class(list[t]) < kRegClasses)
          lvcls = std::max(lvcls, fit_class(list[t]));
      auto class_of = [&](int32_t k) {
        if (wide_ok && !down && up_class(k) >= 0) return up_class(k);
        if (wide_ok && down && down_wide(k)) return kWide;
        return reg_ok && fit_class(k) < kRegClasses ? lvcls : kRegClasses;
      };
      for (int c : {kFat, kWide, kRegClasses, lvcls}) {
        Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t t = L.begin; t < L.begin + L.count; ++t) {
          const int32_t k = list[t];
          if (class_of(k) != c) continue;
          cs.list.push_back(k);
          S.count++;
          S.maxN = std::max(S.maxN, p->N[k]);
          S.maxA = std::max(S.maxA, p->J[k] - p->N[k]);
          S.maxJ = std::max(S.maxJ, p->J[k]);
          const double Nn = p->N[k], Jn = p->J[k], An = Jn - Nn;
          S.p += Nn * Jn - Nn * (Nn - 1) / 2;
          S.u += An * (An + 1) / 2;
          S.n3 += Nn * Nn * Nn;
          S.n2a += Nn * Nn * An;
          S.na2 += Nn * An * An;
          S.a3 += An * An * An;
        }
        if (!S.count) continue;
        ClassSeg g{S, l, c};
        if (c == kWide || c == kFat) number_tiles(cs, g);
        cs.segs.push_back(g);
      }
    }
  };
  make_classes(p->up_list, p->up_levels, false, false, p->cs_factor, true);
  // Schedules for work with no dependence between fronts: the register
  // fronts run in one launch per class over all supernodes (longest first)
  // instead of level by level; fronts beyond the register classes run
  // likewise, longest first, in launches whose workgroup scratch stays
  // within kFlatScratch doubles (a launch holds at least one front).
  // by_a: order A (the inverse of V_s, roots skipped), else J.
  auto make_flat = [&](bool by_a, Op op, ClassSched& cs) {
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    cs.list.reserve(ns);
    // the completion's wide and fat fronts (above the wide threshold) run
    // tile-parallel, in one segment of their own; the inverse of V_s for
    // A > big_a likewise (segment class kBigV)
    const bool fat_ok = op == OP_COMPLETION;
    auto fat = [&](int32_t k) {
      return (fat_ok && is_wide(k)) || (by_a && p->J[k] - p->N[k] > p->big_a);
    };
    auto order = [&](int32_t k) { return by_a ? p->J[k] - p->N[k] : p->J[k]; };
    auto fit = [&](int32_t k) {
      int c = 0;
      while (c < kRegClasses && order(k) > kRegMax[c]) ++c;
      return c;
    };
    auto wanted = [&](int32_t k) { return (!by_a || p->J[k] > p->N[k]) && !fat(k); };
    auto add_front = [&](Level& S, int32_t k) {
      cs.list.push_back(k);
      S.count++;
      S.maxN = std::max(S.maxN, p->N[k]);
      S.maxA = std::max(S.maxA, p->J[k] - p->N[k]);
      S.maxJ = std::max(S.maxJ, p->J[k]);
      const double Nn = p->N[k], Jn = p->J[k], An = Jn - Nn;
      S.p += Nn * Jn - Nn * (Nn - 1) / 2;
      S.u += An * (An + 1) / 2;
      S.n3 += Nn * Nn * Nn;
      S.n2a += Nn * Nn * An;
      S.na2 += Nn * An * An;
      S.a3 += An * An * An;
    };
    for (int c = kRegClasses - 1; c >= 0; --c) {
      std::vector<int32_t> fr;
      for (int32_t k = 0; k < ns; ++k)
        if (wanted(k) && fit(k) == c) fr.push_back(k);
      std::stable_sort(fr.begin(), fr.end(), [&](int32_t x, int32_t y) { return order(x) > order(y); });
      Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t k : fr) add_front(S, k);
      if (S.count) cs.segs.push_back(ClassSeg{S, -1, c});
    }
    {
      std::vector<int32_t> fr;
      for (int32_t k = 0; k < ns; ++k)
        if (wanted(k) && fit(k) == kRegClasses) fr.push_back(k);
      std::stable_sort(fr.begin(), fr.end(), [&](int32_t x, int32_t y) { return order(x) > order(y); });
      Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t k : fr) {
        Level T = S;
        T.count++;
        T.maxN = std::max(T.maxN, p->N[k]);
        T.maxA = std::max(T.maxA, p->J[k] - p->N[k]);
        T.maxJ = std::max(T.maxJ, p->J[k]);
        if (S.count && int64_t(T.count) * slot_doubles(op, T) > kFlatScratch) {
          cs.segs.push_back(ClassSeg{S, -1, kRegClasses});
          S = Level{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        }
        add_front(S, k);
      }
      if (S.count) cs.segs.push_back(ClassSeg{S, -1, kRegClasses});
    }
    {
      // longest first; the completion's in launches of at most
      // kFlatScratchFat doubles of scratch (its slot grows with N and A),
      // the inverse's (no scratch) in one
      std::vector<int32_t> fr;
      for (int32_t k = 0; k < ns; ++k)
        if (fat(k)) fr.push_back(k);
      // the completion's fronts by decreasing N first: its per-front
      // Cholesky of the N x N block steps through the segment's largest N,
      // so the few fronts with many columns share segments of their own
      std::stable_sort(fr.begin(), fr.end(), [&](int32_t x, int32_t y) {
        if (!by_a && p->N[x] != p->N[y]) return p->N[x] > p->N[y];
        return order(x) > order(y);
      });
      const int cls = by_a ? kBigV : kFat;
      auto close_seg = [&](Level& S) {
        if (!S.count) return;
        ClassSeg g{S, -1, cls};
        number_tiles(cs, g);
        cs.segs.push_back(g);
        S = Level{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      };
      Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t k : fr) {
        Level T = S;
        T.count++;
        T.maxN = std::max(T.maxN, p->N[k]);
        T.maxA = std::max(T.maxA, p->J[k] - p->N[k]);
        T.maxJ = std::max(T.maxJ, p->J[k]);
        if (!by_a && S.count && int64_t(T.count) * slot_doubles(op, T) > kFlatScratchFat) close_seg(S);
        add_front(S, k);
      }
      close_seg(S);
    }
  };
  // V_s^-1 needs only V_s; the completion's sweeps need only S and V_s,
  // which a gather pass puts in place beforehand.
  make_flat(true, OP_VINV, p->cs_vinv);
  for (ClassSeg& g : p->cs_vinv.segs)
    if (g.cls == kBigV) {
      const int steps = (g.lv.maxA + 63) / 64 + 2;
      auto a_of = [&](int32_t t) { return p->J[p->cs_vinv.list[t]] - p->N[p->cs_vinv.list[t]]; };
      bool sorted = true;
      for (int32_t t = g.lv.begin + 1; t < g.lv.begin + g.lv.count; ++t) sorted = sorted && a_of(t) <= a_of(t - 1);
      // the length of the prefix with A > 64 q (every front when the list
      // were not in decreasing order of A)
      g.acnt.assign(size_t(steps), g.lv.count);
      if (sorted)
        for (int q = 0; q < steps; ++q) {
          int32_t c = 0;
          while (c < g.lv.count && a_of(g.lv.begin + c) > 64 * q) ++c;
          g.acnt[size_t(q)] = c;
        }
    }
  make_flat(false, OP_COMPLETION, p->cs_compl_flat);
  // the A^3 of the completion's fronts with A > big_a belongs to the
  // tile-parallel factorization that precedes its per-front launches
  for (ClassSeg& g : p->cs_compl_flat.segs)
    for (int32_t t = g.lv.begin; t < g.lv.begin + g.lv.count; ++t) {
      const int32_t k = p->cs_compl_flat.list[t];
      const double An = p->J[k] - p->N[k];
      if (An > p->big_a) g.lv.a3 -= An * An * An;
    }
  // the completion factors the blocks S_AA with A > big_a tile-parallel
  // before its per-front launches: the inverse's segment of those fronts
  {
    ClassSched& cs = p->cs_bigv;
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    for (const ClassSeg& g : p->cs_vinv.segs)
      if (g.cls == kBigV) {
        ClassSeg h = g;
        h.lv.begin = int32_t(cs.list.size());
        h.aa_off = h.an_off = h.nn_off = 0;
        cs.list.insert(cs.list.end(), p->cs_vinv.list.begin() + g.lv.begin,
                       p->cs_vinv.list.begin() + g.lv.begin + g.lv.count);
        cs.segs.push_back(h);
      }
  }
  // The inverse Hessian's steps 1+2 read T_{A_s A_s}, which a gather pass
  // puts in place, so its fronts are independent too.  Wide fronts and the
  // other fronts above kDownRegMaxJ that are not roots take the
  // tile-parallel kernels, the others the register kernels of their order
  // (blocked above order 192); fronts of one kind run together, longest
  // first, in launches of at most kFlatScratch doubles of workgroup scratch.
  {
    ClassSched& cs = p->cs_ihd_flat;
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    cs.list.reserve(ns);
    auto kind = [&](int32_t k) {
      // wide fronts, and every front above the register kernels' order of
      // the root-to-leaf sweeps that is not a root, on the tile-parallel
      // kernels: all fronts run at once here, and one workgroup per front
      // and right-hand side left the chip mostly idle on the 40^3 grid
      // (9,300 fronts of order 65-192, 38 ms for 16 right-hand sides)
      if (is_wide(k) || (p->J[k] > kDownRegMaxJ && p->J[k] != p->N[k])) return kFat;
      int c = 0;
      while (c < kRegClasses && p->J[k] > kRegMax[c]) ++c;
      return c;
    };
    for (int c : {kFat, 5, 4, 3, 2, 1, 0}) {
      std::vector<int32_t> fr;
      for (int32_t k = 0; k < ns; ++k)
        if (kind(k) == c) fr.push_back(k);
      std::stable_sort(fr.begin(), fr.end(), [&](int32_t x, int32_t y) { return p->J[x] > p->J[y]; });
      Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int32_t k : fr) {
        Level T = S;
        T.count++;
        T.maxN = std::max(T.maxN, p->N[k]);
        T.maxA = std::max(T.maxA, p->J[k] - p->N[k]);
        T.maxJ = std::max(T.maxJ, p->J[k]);
        if (S.count && int64_t(T.count) * slot_doubles(OP_IHDOWN, T) > kFlatScratch) {
          ClassSeg g{S, -1, c};
          if (c == kFat) number_tiles(cs, g);
          cs.segs.push_back(g);
          S = Level{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
          T = S;
          T.count = 1;
          T.maxN = p->N[k];
          T.maxA = p->J[k] - p->N[k];
          T.maxJ = p->J[k];
        }
        const double Nn = p->N[k], Jn = p->J[k], An = Jn - Nn;
        T.p += Nn * Jn - Nn * (Nn - 1) / 2;
        T.u += An * (An + 1) / 2;
        T.n3 += Nn * Nn * Nn;
        T.n2a += Nn * Nn * An;
        T.na2 += Nn * An * An;
        T.a3 += An * An * An;
        cs.list.push_back(k);
        S = T;
      }
      if (S.count) {
        ClassSeg g{S, -1, c};
        if (c == kFat) number_tiles(cs, g);
        cs.segs.push_back(g);
      }
    }
  }
  // The Hessian factor's conversions (both directions) touch one front at
  // a time: every supernode, blocked kernel, longest first.
  {
    ClassSched& cs = p->cs_hfac;
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    std::vector<int32_t> fr(static_cast<size_t>(ns));
    for (int32_t k = 0; k < ns; ++k) fr[size_t(k)] = k;
    std::stable_sort(fr.begin(), fr.end(), [&](int32_t x, int32_t y) { return p->J[x] > p->J[y]; });
    Level S{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t k : fr) {
      Level T = S;
      T.count++;
      T.maxN = std::max(T.maxN, p->N[k]);
      T.maxA = std::max(T.maxA, p->J[k] - p->N[k]);
      T.maxJ = std::max(T.maxJ, p->J[k]);
      if (S.count && int64_t(T.count) * slot_doubles(OP_HFAC, T) > kFlatScratch) {
        cs.segs.push_back(ClassSeg{S, -1, kRegClasses});
        S = Level{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        T = S;
        T.count = 1;
        T.maxN = p->N[k];
        T.maxA = p->J[k] - p->N[k];
        T.maxJ = p->J[k];
      }
      const double Nn = p->N[k], Jn = p->J[k], An = Jn - Nn;
      T.p += Nn * Jn - Nn * (Nn - 1) / 2;
      T.u += An * (An + 1) / 2;
      T.n3 += Nn * Nn * Nn;
      T.n2a += Nn * Nn * An;
      T.na2 += Nn * An * An;
      T.a3 += An * An * An;
      cs.list.push_back(k);
      S = T;
    }
    if (S.count) cs.segs.push_back(ClassSeg{S, -1, kRegClasses});
  }
  make_classes(p->down_list, p->down_levels, false, true, p->cs_down, true);
  // the Hessian's steps 2-3: non-root fronts above kDownRegMaxJ on the
  // tile-parallel kernels too (on the 40^3 grid's relaxed plans, thousands
  // of fronts of order 65-192 per sweep, one workgroup per front and
  // right-hand side on the blocked kernel otherwise)
  mid_wide = true;
  make_classes(p->down_list, p->down_levels, false, true, p->cs_hdown, true);
  mid_wide = false;
  p->hd_root = -1;
  p->ihd_root = -1;
  if (!p->down_levels.empty() && p->down_levels[0].count == 1) {
    const int32_t s = p->down_list[p->down_levels[0].begin];
    if (p->J[s] == p->N[s] && p->N[s] > kDownRegMaxJ && !is_wide(s)) {
      p->hd_root = s;
      auto& sg = p->cs_hdown.segs;
      sg.erase(std::remove_if(sg.begin(), sg.end(), [](const ClassSeg& g) { return g.level == 0; }), sg.end());
      // likewise the inverse Hessian's steps 1+2 for that front (its own
      // segment of the all-fronts schedule: the only front of its kind there)
      auto& sh = p->cs_ihd_flat.segs;
      const size_t before = sh.size();
      sh.erase(std::remove_if(sh.begin(), sh.end(),
                              [&](const ClassSeg& g) {
                                return g.lv.count == 1 && p->cs_ihd_flat.list[g.lv.begin] == s;
                              }),
               sh.end());
      p->ihd_root = sh.size() < before ? s : -1;
    }
  }

  // Source offsets of the packed update-block entries: entry (x, y) of
  // supernode s's A_s x A_s block is S(A_s[x], A_s[y]), which lies in the
  // parent's CCS columns when A_s[y] is one of the parent's own columns and
  // in the parent's block otherwise (parents come first in down_list).
  p->gmap.clear();
  if (!(flags & MFB_PLAN_NO_GATHER_MAP) && p->update_doubles <= kGatherMapMax) {
    p->gmap.assign(size_t(p->update_doubles), 0);
    auto pkh = [](int64_t x, int64_t y, int64_t A) { return y * (2 * A - y - 1) / 2 + x; };
    for (int32_t t = 0; t < ns; ++t) {
      const int32_t s = p->down_list[t];
      const int32_t A = p->J[s] - p->N[s];
      if (A == 0) continue;
      const int32_t q = p->parent[s];
      const int32_t Nq = p->N[q], Aq = p->J[q] - Nq;
      const int32_t* rl = &p->rel[p->relbase[s]];
      const int64_t* colq = &p->col[p->colbase[q]];
      for (int32_t y = 0; y < A; ++y)
        for (int32_t x = y; x < A; ++x) {
          const int32_t rx = rl[x], ry = rl[y];
          p->gmap[p->arena[s] + pkh(x, y, A)] =
              ry < Nq ? colq[ry] + (rx - ry) : p->gmap[p->arena[q] + pkh(rx - Nq, ry - Nq, Aq)];
        }
    }
  }
  p->all_levels.assign(1, Level{0, ns, 0, 0, 0, 0, double(p->update_doubles), 0, 0, 0, 0});
  // The gather without the map: one launch per root-to-leaf level over the
  // 64 x 64 lower tiles of every A x A block of the level.
  {
    ClassSched& cs = p->cs_gather;
    cs.list.clear();
    cs.segs.clear();
    cs.pre.clear();
    for (int32_t l = 0; l < int32_t(p->down_levels.size()); ++l) {
      const Level& L = p->down_levels[l];
      Level S{int32_t(cs.list.size()), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      ClassSeg g{S, l, kWide};
      g.aa_off = int32_t(cs.pre.size());
      int32_t acc = 0;
      for (int32_t t = L.begin; t < L.begin + L.count; ++t) {
        const int32_t k = p->down_list[t];
        const int32_t A = p->J[k] - p->N[k];
        if (A == 0) continue;
        cs.list.push_back(k);
        cs.pre.push_back(acc);
        const int32_t nt = (A + kWideTile - 1) / kWideTile;
        acc += nt * (nt + 1) / 2;
        g.lv.count++;
        g.lv.maxA = std::max(g.lv.maxA, A);
        g.lv.u += double(A) * (A + 1) / 2;
      }
      if (!g.lv.count) {
        cs.pre.resize(size_t(g.aa_off));
        continue;
      }
      cs.pre.push_back(acc);
      g.n_aa = acc;
      cs.segs.push_back(g);
    }
  }

  // Partial-product offsets of the wide fronts with at most kPartN columns.
  p->poff.assign(size_t(ns), -1);
  p->part_doubles = 0;
  for (int32_t k = 0; k < ns; ++k) {
    const int32_t A = p->J[k] - p->N[k];
    if (!is_wide(k) || p->N[k] > kPartN || A == 0) continue;
    const int64_t ta = (A + kWideTile - 1) / kWideTile;
    p->poff[size_t(k)] = p->part_doubles;
    p->part_doubles += ta * (ta + 1) * kWideTile * p->N[k];
  }

  // Canonical algorithmic flop counts per supernode (LAPACK conventions).
  for (int32_t k = 0; k < ns; ++k) {
    const double Nn = p->N[k], An = p->J[k] - p->N[k];
    p->fl_factor += Nn * Nn * Nn / 3 + Nn * Nn * An + Nn * An * An;
    p->fl_projinv += 2 * Nn * Nn * Nn / 3 + 2 * An * An * Nn + An * Nn * Nn;
    p->fl_hess += 6 * An * An * Nn + 6 * An * Nn * Nn + 3 * Nn * Nn * Nn;
    p->fl_invhess += 7 * An * An * Nn + 7 * An * Nn * Nn + 3 * Nn * Nn * Nn;
    p->fl_invhess_x += An * An * An / 3;
    p->fl_completion += An * An * An / 3 + 2 * An * An * Nn + An * Nn * Nn + Nn * Nn * Nn;
    p->fl_product += Nn * Nn * Nn / 3 + Nn * Nn * An + Nn * An * An;
    // canonical doubles moved (panel entries pe, packed update entries ue)
    const double pe = Nn * (Nn + An) - Nn * (Nn - 1) / 2, ue = An * (An + 1) / 2;
    p->by_factor += 8 * (2 * pe + 2 * ue);
    p->by_projinv += 8 * (2 * pe + 2 * ue);
    p->by_hess += 8 * (6 * pe + 5 * ue);
    p->by_invhess += 8 * (7 * pe + 7 * ue);
    p->by_completion += 8 * (4 * pe + 5 * ue);
    p->by_product += 8 * (2 * pe + 2 * ue);
  }
  p->colptr_h.assign(cp, cp + n + 1);
  p->rowind_h.assign(ri, ri + p->nnz);
  p->nnz_user = p->nnz;
  return MFB_OK;
}

// Relaxed supernodes (the amalgamation mentioned in Section 8).  Bottom-up
// over the fundamental clique tree, a parent absorbs the child whose merge
// adds the fewest explicit zeros, as long as the merged supernode's zeros
// (its own and those it inherited) stay within `frac` of its entries.  A
// group of G columns whose top supernode has ancestors A is made a dense
// trapezoid: each of its columns holds the group's later columns and A, so
// it has G(G+1)/2 + G A entries whatever the labels, and merging child c
// (G_c columns, ancestors A_c) into p adds G_c |J_p| - G_c |A_c| zeros.
// The union V' of the trapezoids and V is filled in the same order (A_c
// lies inside J_p), and the groups partition it into supernodes: the plan
// is that of V' on this partition; the caller's arrays stay on V and are
// mapped in and out by the entry points.
mfb_status_t build_plan_relaxed(int64_t n, const int64_t* cp, const int32_t* ri, uint32_t flags, double frac,
                                mfb_plan_s* p, const PlanTuning& tune) {
  if (!(frac >= 0.0 && frac < 1.0)) return MFB_EINVAL;
  mfb_plan_s f;
  mfb_status_t st = build_plan(n, cp, ri, flags, &f);
  if (st) return st;
  const int32_t ns = f.ns;
  std::vector<int32_t> into(ns, -1);
  std::vector<int64_t> cols(ns), zeros(ns, 0);
  for (int32_t s = 0; s < ns; ++s) cols[s] = f.N[s];
  for (int32_t s = 0; s < ns; ++s) {  // postorder: the children's groups are final
    const int64_t Js = f.J[s], As = f.J[s] - f.N[s];
    int32_t best = -1;
    int64_t bz = 0;
    for (int32_t q = f.cptr[s]; q < f.cptr[s + 1]; ++q) {
      const int32_t c = f.cidx[q];
      const int64_t Ac = f.J[c] - f.N[c];
      const int64_t z = zeros[c] + zeros[s] + cols[c] * (Js - Ac);
      const double Nm = double(cols[c] + cols[s]);
      if (double(z) <= frac * (Nm * (Nm + 1) / 2 + Nm * double(As)) && (best < 0 || z < bz)) {
        best = c;
        bz = z;
      }
    }
    if (best >= 0) {
      into[best] = s;
      cols[s] += cols[best];
      zeros[s] = bz;
    }
  }
  std::vector<int32_t> top(ns);
  for (int32_t s = ns - 1; s >= 0; --s) top[s] = into[s] < 0 ? s : top[into[s]];
  // members of every group in ascending column order
  std::vector<int64_t> gptr(size_t(ns) + 1, 0);
  for (int64_t v = 0; v < n; ++v) gptr[size_t(top[f.snode_of[v]]) + 1]++;
  for (int32_t s = 0; s < ns; ++s) gptr[s + 1] += gptr[s];
  std::vector<int32_t> mem(static_cast<size_t>(n));
  {
    std::vector<int64_t> fill(gptr.begin(), gptr.end() - 1);
    for (int64_t v = 0; v < n; ++v) mem[size_t(fill[top[f.snode_of[v]]]++)] = int32_t(v);
  }
  // V': column mem[g][i] holds rows mem[g][i..] followed by A of the group's top
  std::vector<int64_t> cp2(static_cast<size_t>(n) + 1, 0);
  for (int32_t g = 0; g < ns; ++g) {
    if (top[g] != g) continue;
    const int64_t G = gptr[g + 1] - gptr[g], a = f.J[g] - f.N[g];
    for (int64_t i = 0; i < G; ++i) cp2[size_t(mem[size_t(gptr[g] + i)]) + 1] = G - i + a;
  }
  for (int64_t v = 0; v < n; ++v) cp2[size_t(v) + 1] += cp2[size_t(v)];
  const int64_t nnz2 = cp2[size_t(n)];
  if (nnz2 - cp[n] >= (int64_t(1) << 31)) return MFB_EINVAL;
  std::vector<int32_t> ri2(static_cast<size_t>(std::max<int64_t>(1, nnz2)));
  for (int32_t g = 0; g < ns; ++g) {
    if (top[g] != g) continue;
    const int64_t G = gptr[g + 1] - gptr[g], a = f.J[g] - f.N[g];
    const int32_t* Ag = ri + cp[f.rep[g]] + f.N[g];
    if (a > 0 && mem[size_t(gptr[g + 1] - 1)] >= Ag[0]) return MFB_ENOTCHORDAL;
    for (int64_t i = 0; i < G; ++i) {
      int64_t o = cp2[size_t(mem[size_t(gptr[g] + i)])];
      for (int64_t t = i; t < G; ++t) ri2[size_t(o++)] = mem[size_t(gptr[g] + t)];
      for (int64_t t = 0; t < a; ++t) ri2[size_t(o++)] = Ag[t];
    }
  }
  // V inside V': shift of every entry, and the entries of V' \ V
  std::vector<int32_t> shift(static_cast<size_t>(std::max<int64_t>(1, cp[n])));
  std::vector<int64_t> zpos;
  zpos.reserve(size_t(nnz2 - cp[n]));
  for (int64_t v = 0; v < n; ++v) {
    int64_t e = cp[v];
    for (int64_t q = cp2[size_t(v)]; q < cp2[size_t(v) + 1]; ++q) {
      if (e < cp[v + 1] && ri[e] == ri2[size_t(q)]) {
        shift[size_t(e)] = int32_t(q - e);
        ++e;
      } else {
        zpos.push_back(q);
      }
    }
    if (e != cp[v + 1]) return MFB_ENOTCHORDAL;  // V is not inside V'
  }
  // the merged groups are the partition of V' (Algorithm 6.1 on V' could
  // pair a parent with another child of equal degree: a supernode need not
  // be a range of labels, and a merged child may sit inside its parent's
  // label range)
  if ((st = validate(n, cp2.data(), ri2.data()))) return st;
  std::vector<int32_t> gid(ns, -1);
  std::vector<std::vector<int32_t>> groups;
  for (int32_t g = 0; g < ns; ++g)
    if (top[g] == g) {
      gid[g] = int32_t(groups.size());
      groups.emplace_back(mem.begin() + gptr[g], mem.begin() + gptr[g + 1]);
    }
  std::vector<int32_t> gpar(groups.size(), -1);
  for (int32_t g = 0; g < ns; ++g)
    if (top[g] == g && f.parent[g] >= 0) gpar[size_t(gid[g])] = gid[top[f.parent[g]]];
  if ((st = finish_plan(n, cp2.data(), ri2.data(), flags, tune, groups, gpar, p))) return st;
  p->relaxed = true;
  p->relax_frac = frac;
  p->nnz_user = cp[n];
  p->vshift = std::move(shift);
  p->zpos = std::move(zpos);
  p->ucolptr_h.assign(cp, cp + n + 1);
  return MFB_OK;
}

}  // namespace mfb
