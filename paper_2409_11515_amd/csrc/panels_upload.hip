// Upload of one triangular solve's schedule into a device workspace.

#include "panels_upload.hpp"

#include <string>

namespace condest {

int tri_upload(char* ws, const size_t* off, const PanelCsr& t, int K, hipStream_t s, DevTri& out) {
  auto up = [&](int slot, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(ws + off[slot], src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  hipError_t e = up(kOffRp, t.off_rp.data(), (t.n + 1) * 8);
  if (e == hipSuccess) e = up(kOffCol, t.off_col.data(), t.off_col.size() * 4);
  if (e == hipSuccess) e = up(kOffVal, t.off_val.data(), t.off_val.size() * 8);
  if (e == hipSuccess) e = up(kOffSplit, t.off_split.data(), static_cast<size_t>(t.n) * 8);
  if (e == hipSuccess) e = up(kWinv, t.winv.data(), t.winv.size() * 8);
  if (e == hipSuccess) e = up(kWoff, t.woff.data(), t.woff.size() * 8);
  if (e == hipSuccess) e = up(kTaskRec, t.task_rec.data(), t.task_rec.size() * 4);
  if (e == hipSuccess) e = up(kTaskRp, t.task_rp.data(), t.task_rp.size() * 8);
  if (e == hipSuccess) e = up(kTaskSp, t.task_sp.data(), t.task_sp.size() * 8);
  if (e == hipSuccess) e = up(kSlotGroup, t.slot_group.data(), t.slot_group.size() * 4);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("solve upload: ") + hipGetErrorString(e));
  auto at = [&](int slot) { return ws + off[slot]; };
  if (t.nslots > 0)
    launch_fill(static_cast<long long>(t.nslots) * t.prows * K, reinterpret_cast<double*>(at(kPartials)), kPending, s);
  out.n = t.n;
  out.prows = t.prows;
  out.off_rp = reinterpret_cast<const long long*>(at(kOffRp));
  out.off_col = reinterpret_cast<const int*>(at(kOffCol));
  out.off_val = reinterpret_cast<const double*>(at(kOffVal));
  out.off_split = reinterpret_cast<const long long*>(at(kOffSplit));
  out.winv = reinterpret_cast<const double*>(at(kWinv));
  out.woff = reinterpret_cast<const long long*>(at(kWoff));
  out.partials = reinterpret_cast<double*>(at(kPartials));
  out.task_rec = reinterpret_cast<const int*>(at(kTaskRec));
  out.task_rp = reinterpret_cast<const long long*>(at(kTaskRp));
  out.task_sp = reinterpret_cast<const long long*>(at(kTaskSp));
  out.slot_group = t.slot_group.empty() ? nullptr : reinterpret_cast<const int*>(at(kSlotGroup));
  out.ntasks = static_cast<int>(t.task_panel.size());
  for (int l = 0; l <= kTaskLists; ++l) out.list_off[l] = t.list_off[l];
  return COND_OK;
}

}  // namespace condest
