// Work lists of a batch context: host-built tables of (instance, index)
// pairs that the batched kernels read by workgroup index.  A sample tile
// (i, t) covers samples t*tile .. t*tile + tile - 1 of instance i; a row tile
// (i, b) covers rows b*rpb .. b*rpb + rpb - 1 of instance i's update.  The
// kernels trust these tables (an instance index past the descriptor table or
// a row past an instance's T*m reads and writes another instance's memory),
// so every table is built and checked here, on the host, before it is
// uploaded.  Host-only C++ (no HIP), so the checks also run without a GPU.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace mppi {

struct WorkItem {
  int32_t inst, idx;  // the layout of HIP's int2, as the kernels read it
};

// Sample tiles of `tile` samples for instances with K[i] samples and
// horizon T[i], the longest horizon first (stable: instance order within a
// horizon), so the dispatcher starts the long rollouts early.
inline std::vector<WorkItem> build_sample_tiles(const int32_t* K, const int32_t* T, int n_inst,
                                                int tile) {
  std::vector<int> order(n_inst);
  for (int i = 0; i < n_inst; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return T[a] > T[b]; });
  std::vector<WorkItem> out;
  for (int i : order)
    for (int t = 0; static_cast<int64_t>(t) * tile < K[i]; ++t) out.push_back(WorkItem{i, t});
  return out;
}

// Row tiles of `rows_per_block` rows for instances with TM[i] = T*m rows.
inline std::vector<WorkItem> build_row_tiles(const int32_t* TM, int n_inst, int rows_per_block) {
  std::vector<WorkItem> out;
  for (int i = 0; i < n_inst; ++i)
    for (int b = 0; static_cast<int64_t>(b) * rows_per_block < TM[i]; ++b)
      out.push_back(WorkItem{i, b});
  return out;
}

// Checks a table of n_items entries against the instances' extents
// (samples for sample tiles, rows for row tiles) and the table's capacity in
// the workspace: every instance index is in [0, n_inst), every entry starts
// inside its instance (idx >= 0, idx * unit < extent), and every instance's
// units are covered exactly once (ceil(extent / unit) distinct entries).
// Returns an empty string when the table is valid, else the first problem.
inline std::string check_work_list(const WorkItem* items, int64_t n_items, int64_t capacity,
                                   int unit, const int32_t* extent, int n_inst) {
  char buf[160];
  if (unit < 1) return "work unit must be positive";
  if (n_inst < 1) return "no instances";
  if (n_items < 0 || n_items > capacity) {
    snprintf(buf, sizeof buf, "%lld entries for a table of %lld", static_cast<long long>(n_items),
             static_cast<long long>(capacity));
    return buf;
  }
  std::vector<int64_t> offset(n_inst + 1, 0);
  for (int i = 0; i < n_inst; ++i) {
    if (extent[i] < 1) {
      snprintf(buf, sizeof buf, "instance %d has extent %d", i, extent[i]);
      return buf;
    }
    offset[i + 1] = offset[i] + (extent[i] + unit - 1) / unit;
  }
  if (offset[n_inst] != n_items) {
    snprintf(buf, sizeof buf, "%lld entries, the instances need %lld",
             static_cast<long long>(n_items), static_cast<long long>(offset[n_inst]));
    return buf;
  }
  std::vector<char> seen(static_cast<size_t>(n_items), 0);
  for (int64_t q = 0; q < n_items; ++q) {
    const WorkItem w = items[q];
    if (w.inst < 0 || w.inst >= n_inst) {
      snprintf(buf, sizeof buf, "entry %lld: instance %d of %d", static_cast<long long>(q), w.inst,
               n_inst);
      return buf;
    }
    if (w.idx < 0 || static_cast<int64_t>(w.idx) * unit >= extent[w.inst]) {
      snprintf(buf, sizeof buf, "entry %lld: index %d x %d outside instance %d's extent %d",
               static_cast<long long>(q), w.idx, unit, w.inst, extent[w.inst]);
      return buf;
    }
    char& s = seen[static_cast<size_t>(offset[w.inst] + w.idx)];
    if (s) {
      snprintf(buf, sizeof buf, "entry %lld: instance %d index %d listed twice",
               static_cast<long long>(q), w.inst, w.idx);
      return buf;
    }
    s = 1;
  }
  return "";
}

}  // namespace mppi
