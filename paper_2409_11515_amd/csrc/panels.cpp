// Panel schedules of the sparse triangular solves: the planner (panel cuts
// chosen by a measured cost model, dependency levels, slices of heavy panels,
// task records), the inverses of the panel triangles, the schedule of
// several independent blocks joined into one, the host replay of a solve,
// and the device layout of one solve. Plain host C++.

#include "panels.hpp"

#include <algorithm>
#include <string>

namespace condest {

namespace {

// A panel whose rows hold more off-panel entries than this is cut into
// slices (at most kMaxSlices) that separate blocks sum in parallel. The
// slices take a row's entries on rows more than one panel height (prows)
// before the panel; the finish step takes the newer ones, so a chain of
// panels (a dense separator block) waits for its predecessor in one step,
// not two.
constexpr int64_t kSliceEntries = 4096;
constexpr int32_t kMaxSlices = kMaxSlicesDev;

// Panel boundaries: a panel closes when it holds prows rows, or -- once
// it holds at least kMinPanelRows -- before a row that needs nothing inside
// it. Such a row usually opens an independent subtree of the elimination
// order (a new leaf of the nested dissection); cutting there keeps independent
// subtrees in different panels, so they are solved in parallel instead of as
// a chain. With `merge`, such a row instead joins the open panel when it reads
// panels exactly as deep as the open panel does: it would run in the same
// dependency level anyway, and one task fewer is cheaper than the parallelism
// (the leaves of a nested dissection are thousands of panels of a few rows).
// A panel also closes at a kPanel-row boundary when the next row reads a
// panel that is deeper in the dependency order than anything the open panel
// reads, so that the rows before do not wait for it. What remains inside a
// panel are chains (a dense separator block, mostly), which one block solves
// at once with the inverse of the panel's triangle.
constexpr int32_t kMinPanelRows = 4;

std::vector<int32_t> cut_panels(const HostCsr& t, bool merge, int32_t prows) {
  std::vector<int32_t> ps{0};
  std::vector<int32_t> pid(t.n, 0), plevel;  // panel of each closed row, level of each panel
  int32_t s = 0;
  // 1 + the deepest closed panel that row e reads (columns left of the open panel)
  auto ext_level = [&](int32_t e) {
    int32_t lv = 0;
    for (int64_t p = t.rowptr[e]; p < t.rowptr[e + 1]; ++p)
      if (t.col[p] < s) lv = std::max(lv, plevel[pid[t.col[p]]] + 1);
    return lv;
  };
  int32_t cur = t.n ? ext_level(0) : 0;
  for (int32_t e = 1; e < t.n; ++e) {
    bool needs_panel = false;
    for (int64_t p = t.rowptr[e]; p < t.rowptr[e + 1] && !needs_panel; ++p)
      needs_panel = t.col[p] >= s;
    const int32_t rows = e - s;
    const int32_t lv = ext_level(e);
    if (rows >= prows || (!needs_panel && rows >= kMinPanelRows && (!merge || lv != cur)) ||
        (rows % kPanel == 0 && lv > cur)) {
      const int32_t q = static_cast<int32_t>(plevel.size());
      for (int32_t i = s; i < e; ++i) pid[i] = q;
      plevel.push_back(cur);
      ps.push_back(e);
      s = e;
      cur = ext_level(e);
    } else {
      cur = std::max(cur, lv);
    }
  }
  ps.push_back(t.n);
  return ps;
}

// Level of each panel: one more than the deepest panel it reads from.
std::vector<int32_t> panel_levels(const HostCsr& t, const std::vector<int32_t>& pstart,
                                  std::vector<int32_t>& pid) {
  const int32_t np = static_cast<int32_t>(pstart.size()) - 1;
  pid.assign(t.n, 0);
  for (int32_t p = 0; p < np; ++p)
    for (int32_t i = pstart[p]; i < pstart[p + 1]; ++i) pid[i] = p;
  std::vector<int32_t> level(np, 0);
  for (int32_t i = 0; i < t.n; ++i)
    for (int64_t p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) {
      const int32_t q = pid[t.col[p]];
      if (q != pid[i]) level[pid[i]] = std::max(level[pid[i]], level[q] + 1);
    }
  return level;
}

int32_t slices_of(int64_t work) {
  return static_cast<int32_t>(std::min<int64_t>(kMaxSlices, (work + kSliceEntries - 1) / kSliceEntries));
}

// Estimated solve time of a cut, in microseconds: every dependency level
// costs a wait-and-publish round trip, every task a fixed hand-out and
// set-up cost spread over the resident blocks. Both constants are a
// least-squares fit to eight measured solves on MI355X (256 resident
// blocks): the four factor orientations of a 242k-row hydro-mechanical
// system, each cut both ways.
constexpr double kLevelUs = 2.5;
constexpr double kTaskUs = 0.0152;

double cut_cost(const HostCsr& t, const std::vector<int32_t>& pstart) {
  std::vector<int32_t> pid;
  const std::vector<int32_t> level = panel_levels(t, pstart, pid);
  const int32_t np = static_cast<int32_t>(pstart.size()) - 1;
  int64_t tasks = 0;
  for (int32_t p = 0; p < np; ++p) {
    int64_t work = 0;  // entries left of the panel
    for (int32_t i = pstart[p]; i < pstart[p + 1]; ++i)
      for (int64_t e = t.rowptr[i]; e < t.rowptr[i + 1]; ++e) work += t.col[e] < pstart[p];
    const int32_t S = slices_of(work);
    tasks += S > 1 ? S + 1 : 1;
  }
  const int32_t levels = np ? 1 + *std::max_element(level.begin(), level.end()) : 0;
  return kLevelUs * levels + kTaskUs * static_cast<double>(tasks);
}

// The device order of the tasks and everything indexed by it: the tasks are
// dealt round-robin to kTaskLists lists in dependency order (so each list is
// in dependency order, and each holds about 1/kTaskLists of every level),
// then the records, row pointers and split points (and, for joined
// schedules, the blocks) are laid out list after list. Built from
// the tasks, panels and inverse offsets alone.
void finish_records(PanelCsr& s) {
  const size_t ntasks = s.task_panel.size();
  s.list_off.assign(kTaskLists + 1, 0);
  for (size_t k = 0; k < ntasks; ++k) ++s.list_off[k % kTaskLists + 1];
  for (int l = 0; l < kTaskLists; ++l) s.list_off[l + 1] += s.list_off[l];
  s.task_slot.assign(ntasks, 0);
  std::vector<int32_t> next(s.list_off.begin(), s.list_off.end() - 1);
  for (size_t k = 0; k < ntasks; ++k) s.task_slot[k] = next[k % kTaskLists]++;
  s.task_rec.assign(8 * ntasks, 0);
  const int32_t R = s.prows;
  s.task_rp.assign(ntasks * (R + 1), 0);
  s.task_sp.assign(ntasks * R, 0);
  for (size_t k = 0; k < ntasks; ++k) {
    const size_t q = static_cast<size_t>(s.task_slot[k]);
    const int32_t p = s.task_panel[k];
    const int64_t w = s.woff.empty() ? 0 : s.woff[p];
    const int32_t lo = s.pstart[p], cnt = s.pstart[p + 1] - lo;
    const int32_t rec[8] = {p, s.task_kind[k], lo, cnt, s.panel_split[p], s.panel_slot[p],
                            static_cast<int32_t>(static_cast<uint32_t>(w & 0xffffffffLL)),
                            static_cast<int32_t>(w >> 32)};
    std::copy(rec, rec + 8, s.task_rec.begin() + 8 * q);
    for (int32_t r = 0; r <= R; ++r) s.task_rp[q * (R + 1) + r] = s.off_rp[lo + std::min(r, cnt)];
    for (int32_t r = 0; r < cnt; ++r) s.task_sp[q * R + r] = s.off_split[lo + r];
  }
  s.slot_group.clear();
  if (s.task_group.empty()) return;
  s.slot_group.assign(ntasks, 0);
  for (size_t k = 0; k < ntasks; ++k) s.slot_group[s.task_slot[k]] = s.task_group[k];
}

}  // namespace

PanelCsr split_panels(const HostCsr& t, int32_t prows) {
  PanelCsr s;
  s.n = t.n;
  s.prows = prows;
  // the cheaper of the two cuts by the cost model (merging the leaves pays
  // where they are many small panels, splitting where they are few)
  std::vector<int32_t> split = cut_panels(t, false, prows), merged = cut_panels(t, true, prows);
  s.pstart = cut_cost(t, merged) < cut_cost(t, split) ? std::move(merged) : std::move(split);
  const int32_t np = static_cast<int32_t>(s.pstart.size()) - 1;
  std::vector<int32_t> pid;
  const std::vector<int32_t> level = panel_levels(t, s.pstart, pid);
  std::vector<int32_t> order(np);
  for (int32_t p = 0; p < np; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return level[a] < level[b]; });
  s.levels = np ? 1 + *std::max_element(level.begin(), level.end()) : 0;
  s.off_rp.assign(t.n + 1, 0);
  s.in_rp.assign(t.n + 1, 0);
  s.off_split.assign(t.n, 0);
  for (int32_t i = 0; i < t.n; ++i) {
    const int32_t lo = s.pstart[pid[i]];
    for (int64_t p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) {
      const int32_t j = t.col[p];
      if (j < lo) {
        s.off_col.push_back(j);
        s.off_val.push_back(t.val[p]);
      } else {
        s.in_col.push_back(j - lo);
        s.in_val.push_back(t.val[p]);
      }
    }
    s.off_rp[i + 1] = static_cast<int64_t>(s.off_col.size());
    s.in_rp[i + 1] = static_cast<int64_t>(s.in_col.size());
  }
  // tasks: whole panels, or slices followed by their finish step
  s.panel_split.assign(np, 1);
  s.panel_slot.assign(np, 0);
  for (int32_t p : order) {
    const int64_t work = s.off_rp[s.pstart[p + 1]] - s.off_rp[s.pstart[p]];
    const int32_t S = slices_of(work);
    if (S <= 1) {
      s.task_panel.push_back(p);
      s.task_kind.push_back(-1);
      s.task_level.push_back(level[p]);
      continue;
    }
    s.panel_split[p] = S;
    s.panel_slot[p] = s.nslots;
    s.nslots += S;
    const int32_t c0 = s.pstart[p] - prows;  // older entries: columns below c0
    for (int32_t i = s.pstart[p]; i < s.pstart[p + 1]; ++i) {
      int64_t e = s.off_rp[i];
      while (e < s.off_rp[i + 1] && s.off_col[e] < c0) ++e;  // columns are sorted in a row
      s.off_split[i] = e;
    }
    for (int32_t k = 0; k <= S; ++k) {
      s.task_panel.push_back(p);
      s.task_kind.push_back(k);
      s.task_level.push_back(level[p]);
    }
  }
  return s;
}

PanelCsr merge_panels(const std::vector<const PanelCsr*>& parts, const std::vector<int64_t>& offsets,
                      const std::vector<int32_t>& groups) {
  PanelCsr m;
  m.prows = parts.empty() ? kPanel : parts[0]->prows;  // the parts share one panel height
  // every array sized once (the joined schedules of a large batch hold
  // billions of entries: no regrowth)
  size_t rows = 0, off = 0, in = 0, panels = 0, winv = 0, tasks = 0;
  for (const PanelCsr* s : parts) {
    rows += static_cast<size_t>(s->n);
    off += s->off_col.size();
    in += s->in_col.size();
    panels += s->pstart.size() - 1;
    winv += s->winv.size();
    tasks += s->task_panel.size();
  }
  m.off_rp.reserve(rows + 1);
  m.in_rp.reserve(rows + 1);
  m.off_split.reserve(rows);
  m.off_col.reserve(off);
  m.off_val.reserve(off);
  m.in_col.reserve(in);
  m.in_val.reserve(in);
  m.pstart.reserve(panels + 1);
  m.panel_split.reserve(panels);
  m.panel_slot.reserve(panels);
  m.woff.reserve(panels);
  m.winv.reserve(winv);
  m.task_panel.reserve(tasks);
  m.task_kind.reserve(tasks);
  m.task_level.reserve(tasks);
  m.task_group.reserve(tasks);
  m.off_rp.push_back(0);
  m.in_rp.push_back(0);
  m.pstart.push_back(0);
  std::vector<int32_t> panel0(parts.size());  // first merged panel of each part
  for (size_t k = 0; k < parts.size(); ++k) {
    const PanelCsr& s = *parts[k];
    const int32_t r0 = static_cast<int32_t>(offsets[k]);
    const int64_t e_off = static_cast<int64_t>(m.off_col.size());
    const int64_t e_in = static_cast<int64_t>(m.in_col.size());
    const int32_t slot0 = m.nslots;
    const int64_t w0 = static_cast<int64_t>(m.winv.size());
    panel0[k] = static_cast<int32_t>(m.pstart.size()) - 1;
    for (int32_t i = 0; i < s.n; ++i) {
      m.off_rp.push_back(e_off + s.off_rp[i + 1]);
      m.in_rp.push_back(e_in + s.in_rp[i + 1]);
      m.off_split.push_back(e_off + s.off_split[i]);
    }
    for (int32_t c : s.off_col) m.off_col.push_back(c + r0);
    m.off_val.insert(m.off_val.end(), s.off_val.begin(), s.off_val.end());
    m.in_col.insert(m.in_col.end(), s.in_col.begin(), s.in_col.end());  // panel-relative
    m.in_val.insert(m.in_val.end(), s.in_val.begin(), s.in_val.end());
    const int32_t np = static_cast<int32_t>(s.pstart.size()) - 1;
    for (int32_t q = 0; q < np; ++q) {
      m.pstart.push_back(r0 + s.pstart[q + 1]);
      m.panel_split.push_back(s.panel_split[q]);
      m.panel_slot.push_back(slot0 + s.panel_slot[q]);
      m.woff.push_back(w0 + s.woff[q]);
    }
    m.winv.insert(m.winv.end(), s.winv.begin(), s.winv.end());
    m.nslots += s.nslots;
    m.levels = std::max(m.levels, s.levels);
    m.n += s.n;
  }
  // tasks of all parts by level; within a level, part by part in their order
  struct Ref {
    int32_t level, part, task;
  };
  std::vector<Ref> refs;
  refs.reserve(tasks);
  for (size_t k = 0; k < parts.size(); ++k)
    for (size_t t = 0; t < parts[k]->task_panel.size(); ++t)
      refs.push_back({parts[k]->task_level[t], static_cast<int32_t>(k), static_cast<int32_t>(t)});
  std::stable_sort(refs.begin(), refs.end(), [](const Ref& a, const Ref& b) { return a.level < b.level; });
  for (const Ref& r : refs) {
    const PanelCsr& s = *parts[r.part];
    m.task_panel.push_back(panel0[r.part] + s.task_panel[r.task]);
    m.task_kind.push_back(s.task_kind[r.task]);
    m.task_level.push_back(r.level);
    m.task_group.push_back(groups[r.part]);
  }
  finish_records(m);
  return m;
}

// The inverse of every panel's triangle: its in-panel entries below the
// diagonal and diag (nullptr: a unit diagonal) on it, inverted column by
// column by substitution in float64 and stored packed by rows. The kernel
// then forms a panel's values as one product with it instead of up to prows
// dependent steps.
void invert_panels(PanelCsr& s, const double* diag) {
  const int32_t np = static_cast<int32_t>(s.pstart.size()) - 1;
  const int32_t R = s.prows;
  s.woff.assign(np, 0);
  int64_t total = 0;
  // each triangle starts on a 16-byte boundary (an even offset): the kernel
  // copies it into LDS 16 bytes per lane, up to one value past its end
  for (int32_t p = 0; p < np; ++p) {
    s.woff[p] = total;
    const int64_t cnt = s.pstart[p + 1] - s.pstart[p];
    total += (cnt * (cnt + 1) / 2 + 1) / 2 * 2;
  }
  s.winv.assign(total, 0.0);
  std::vector<double> t(static_cast<size_t>(R) * R), w(static_cast<size_t>(R) * R);
  for (int32_t p = 0; p < np; ++p) {
    const int32_t lo = s.pstart[p], cnt = s.pstart[p + 1] - lo;
    // the triangle, dense: strictly lower entries, then the diagonal
    std::fill(t.begin(), t.end(), 0.0);
    for (int32_t r = 0; r < cnt; ++r) {
      const int32_t i = lo + r;
      for (int64_t e = s.in_rp[i]; e < s.in_rp[i + 1]; ++e) t[r * R + s.in_col[e]] = s.in_val[e];
      t[r * R + r] = diag ? diag[i] : 1.0;
    }
    std::fill(w.begin(), w.end(), 0.0);
    for (int32_t c = 0; c < cnt; ++c)
      for (int32_t r = c; r < cnt; ++r) {
        double a = r == c ? 1.0 : 0.0;
        for (int32_t k = c; k < r; ++k) a -= t[r * R + k] * w[k * R + c];
        w[r * R + c] = a / t[r * R + r];
      }
    double* out = s.winv.data() + s.woff[p];
    for (int32_t r = 0; r < cnt; ++r)
      for (int32_t c = 0; c <= r; ++c) out[r * (r + 1) / 2 + c] = w[r * R + c];
  }
  finish_records(s);
}

// Row i -> n-1-i and column j -> n-1-j: an upper factor becomes lower.
HostCsr reverse_order(const HostCsr& u) {
  HostCsr r;
  const int32_t n = u.n;
  r.n = n;
  r.rowptr.assign(n + 1, 0);
  r.col.reserve(u.nnz());
  r.val.reserve(u.nnz());
  for (int32_t k = 0; k < n; ++k) {
    const int32_t i = n - 1 - k;
    // walking row i backwards keeps the reversed columns increasing
    for (int64_t p = u.rowptr[i + 1]; p-- > u.rowptr[i];) {
      r.col.push_back(n - 1 - u.col[p]);
      r.val.push_back(u.val[p]);
    }
    r.rowptr[k + 1] = static_cast<int64_t>(r.col.size());
  }
  return r;
}

// One solve as the device runs it, on the host: the tasks in ticket order,
// read from the same task records; a slice task sums its share of each row's
// older off-panel entries into its slot, a finish task adds the slots in
// order and the newest entries, a whole-panel task all off-panel entries;
// then the panel's values are the product with its packed triangle inverse.
// Every value a task reads must have been solved by an earlier ticket (the
// condition under which every wait on the device ends) and every slot a
// finish step reads must have been written; otherwise the schedule is
// reported broken (returns false).
bool replay_solve(const PanelCsr& t, const int32_t* gather, const double* in, double* out) {
  const int32_t n = t.n;
  std::vector<char> ready(n, 0);
  const int32_t R = t.prows;
  std::vector<double> slots(static_cast<size_t>(t.nslots) * R, 0.0);
  std::vector<char> slot_set(static_cast<size_t>(t.nslots) * R, 0);
  std::vector<double> acc(R);
  bool ok = true;
  auto sum = [&](int64_t e0, int64_t e1) {
    double a = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
      ok = ok && ready[t.off_col[e]];
      a += t.off_val[e] * out[t.off_col[e]];
    }
    return a;
  };
  const size_t ntasks = t.task_panel.size();
  for (size_t k = 0; k < ntasks && ok; ++k) {
    const size_t q = static_cast<size_t>(t.task_slot[k]);
    const int32_t* rec = &t.task_rec[8 * q];
    const int32_t kind = rec[1], lo = rec[2], cnt = rec[3], S = rec[4], slot = rec[5];
    const int64_t woff = static_cast<int64_t>(static_cast<uint32_t>(rec[6])) |
                         (static_cast<int64_t>(rec[7]) << 32);
    const int64_t* trp = &t.task_rp[q * (R + 1)];
    const int64_t* tsp = &t.task_sp[q * R];
    if (kind >= 0 && kind < S) {  // slice
      for (int32_t r = 0; r < cnt; ++r) {
        const int64_t q0 = trp[r], len = tsp[r] - q0;
        const size_t at = static_cast<size_t>(slot + kind) * R + r;
        slots[at] = sum(q0 + len * kind / S, q0 + len * (kind + 1) / S);
        slot_set[at] = 1;
      }
      continue;
    }
    for (int32_t r = 0; r < cnt; ++r) {
      const int32_t i = lo + r;
      double sums;
      if (kind < 0) {
        sums = sum(trp[r], trp[r + 1]);
      } else {  // finish
        sums = 0.0;
        for (int32_t m = 0; m < S; ++m) {
          const size_t at = static_cast<size_t>(slot + m) * R + r;
          ok = ok && slot_set[at];
          sums += slots[at];
        }
        sums += sum(tsp[r], trp[r + 1]);
      }
      acc[r] = in[gather ? gather[i] : i] - sums;
    }
    const double* w = t.winv.data() + woff;
    for (int32_t r = 0; r < cnt; ++r) {
      double x = 0.0;
      for (int32_t c = 0; c <= r; ++c) x += w[r * (r + 1) / 2 + c] * acc[c];
      out[lo + r] = x;
      ready[lo + r] = 1;
    }
  }
  for (int32_t i = 0; i < n && ok; ++i) ok = ready[i];
  return ok;
}

void tri_layout(const PanelCsr& t, int K, Layout& L, size_t* o) {
  const size_t n = t.n;
  o[kOffRp] = L.take((n + 1) * 8);
  o[kOffCol] = L.take(t.off_col.size() * 4);
  o[kOffVal] = L.take(t.off_val.size() * 8);
  o[kOffSplit] = L.take(n * 8);
  o[kPartials] = L.take(static_cast<size_t>(t.nslots) * t.prows * K * 8);
  o[kWinv] = L.take(t.winv.size() * 8);
  o[kWoff] = L.take(t.woff.size() * 8);
  o[kTaskRec] = L.take(t.task_rec.size() * 4);
  o[kTaskRp] = L.take(t.task_rp.size() * 8);
  o[kTaskSp] = L.take(t.task_sp.size() * 8);
  o[kSlotGroup] = L.take(t.slot_group.size() * 4);
}

}  // namespace condest
