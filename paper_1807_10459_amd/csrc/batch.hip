// Batch engine behind cmi_ksg_batch, ksg_greedy_step and select_parents: a list of CMI
// problems becomes a plan (host), a descriptor upload and one set of launches on the
// context's stream.
//
//   plan_batch     grouping (problems sharing Y, Z, N, k with 1-D X), key-ordered window sets,
//                  wide problems (17..32 columns), the column pool layout and pack jobs, the
//                  per-problem / per-group / Y/Z descriptors, the work items in XCD-aware
//                  longest-first order, the launch segments and the grouped launch chunks;
//   upload_batch   one pinned staging block, three copies (descriptors, items, pack jobs);
//   enqueue_batch  key orders, pack, optional finite check, group key order + interleave, the
//                  single-problem launches side by side on auxiliary streams, the grouped
//                  chunks (radius, Y/Z counts, X counts), the finalisation.
//
// With KSG_OPT_USE_GRAPH the launches of a batch are captured once into a HIP graph, keyed by
// everything the plan depends on; when the same batch comes again (a greedy step re-run on
// the same columns, a benchmark step) the graph is replayed and the host planning, the upload
// and the per-launch overhead are skipped.  The graph owns private copies of the descriptors,
// items and pack jobs; the work buffers it writes (pool, E, T, partials) are the context's and
// are rewritten by every replay, and a reallocation of any of them retires every graph
// captured before it (freed at the next capture).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"
#include "runtime.h"

using namespace ksg;

namespace {

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int kp_for(int k) { return k + 1 <= 5 ? 5 : (k + 1 <= 9 ? 9 : 17); }

// A unit of scheduling: one problem (ungrouped) or one group, with all its tiles.
struct Unit {
  int id;
  int n_tiles;
  double cost;
};

// Work items for a list of units (already in longest-first order).  With many units, each
// unit goes whole to one of the 8 XCDs (least-loaded first) and the items are interleaved
// so that work-group b, which the dispatcher places on XCD b % 8, takes the next item of
// that XCD's list: a problem's columns are then read into one XCD's L2 only.  Empty slots
// (prob = -1) return at once.  With few units the plain order keeps every XCD busy.
std::vector<WorkItem> order_items(const std::vector<Unit>& units) {
  constexpr int kXcd = 8;
  std::vector<WorkItem> out;
  if ((int)units.size() < 4 * kXcd) {
    for (const Unit& u : units)
      for (int t = 0; t < u.n_tiles; ++t) out.push_back(WorkItem{u.id, t});
    return out;
  }
  std::vector<std::vector<WorkItem>> bins(kXcd);
  std::vector<double> load(kXcd, 0.0);
  for (const Unit& u : units) {
    int x = 0;
    for (int i = 1; i < kXcd; ++i)
      if (load[i] < load[x]) x = i;
    load[x] += u.cost;
    for (int t = 0; t < u.n_tiles; ++t) bins[x].push_back(WorkItem{u.id, t});
  }
  size_t L = 0;
  for (auto& b : bins) L = std::max(L, b.size());
  out.assign(L * kXcd, WorkItem{-1, 0});
  for (int x = 0; x < kXcd; ++x)
    for (size_t s = 0; s < bins[x].size(); ++s) out[s * kXcd + x] = bins[x][s];
  return out;
}

// Problems that share Y, Z, N and k and differ only in a 1-D X column can be searched as a
// group (Y/Z distances computed once per pair for the whole group).
bool groupable(const Problem& p) {
  if (p.dx != 1 || p.dy != 1 || p.dz > kGroupMaxM || p.k + 1 > 9) return false;
  if (p.eps_out || p.counts_out || p.local_out) return false;
  for (int a = 1; a < 2 + p.dz; ++a)
    if (p.perm[a]) return false;
  return true;
}

double brute_cost(const Problem& p) { return (double)p.n * (double)p.n * (4.0 * (p.dx + p.dy + p.dz) + 2.0); }

}  // namespace

int ksg_ctx::validate(const Problem& p, int index) {
  const int D = p.dx + p.dy + p.dz;
  if (p.dx < 1 || p.dy < 1 || p.dz < 0 || D > KSG_MAX_DIMS)
    return fail(KSG_EINVAL, "problem %d: dims (%d,%d,%d) outside d_x>=1, d_y>=1, d_z>=0, sum<=%d",
                index, p.dx, p.dy, p.dz, KSG_MAX_DIMS);
  if (p.k < 1 || p.k > KSG_MAX_K)
    return fail(KSG_EINVAL, "problem %d: k=%d outside [1, %d]", index, p.k, KSG_MAX_K);
  if (algorithm == 2 && D > kMaxDimsCompiled)
    return fail(KSG_EINVAL, "problem %d: %d columns; KSG algorithm 2 supports at most %d", index, D,
                kMaxDimsCompiled);
  if (p.n > (int64_t)INT32_MAX - 1024)
    return fail(KSG_EINVAL, "problem %d: N=%lld too large", index, (long long)p.n);
  if (p.n <= p.k)
    return fail(KSG_ETOOFEW, "problem %d: N=%lld <= k=%d", index, (long long)p.n, p.k);
  for (int a = 0; a < D; ++a)
    if (!p.col[a]) return fail(KSG_EINVAL, "problem %d: null column %d", index, a);
  return KSG_OK;
}

// ============================================================== planning

int ksg_ctx::plan_batch(const std::vector<Problem>& probs, BatchPlan& P) {
  const int np = (int)probs.size();
  P.np = np;
  int64_t nmax = 0;
  for (int i = 0; i < np; ++i) {
    int st = validate(probs[i], i);
    if (st) return st;
    nmax = std::max<int64_t>(nmax, probs[i].n);
  }
  int st = ensure_htab(nmax);
  if (st) return st;

  // ---- grouping: problems with identical (N, k, Y, Z) and 1-D X ----
  std::vector<int> group_of(np, -1);
  std::vector<std::vector<int>> groups;  // member problem indices
  std::vector<int> group_size_of;        // G of each group's kernel
  if (group_size != 0 && algorithm == 1) {
    std::map<std::vector<intptr_t>, std::vector<int>> by_key;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      if (!groupable(p)) continue;
      std::vector<intptr_t> key = {(intptr_t)p.n, p.k, p.dz, (intptr_t)p.col[1]};
      for (int a = 0; a < p.dz; ++a) key.push_back((intptr_t)p.col[2 + a]);
      by_key[key].push_back(i);
    }
    for (auto& kv : by_key) {
      const std::vector<int>& members = kv.second;
      if (members.size() < 2) continue;
      const int m = probs[members[0]].dz;
      int G = group_size > 0 ? group_size : tuned_group_size(m, probs[members[0]].k);
      if (m > kGroupMaxM16) G = 8;  // the wider conditioning sets are compiled for groups of 8
      for (size_t s = 0; s < members.size(); s += G) {
        std::vector<int> g(members.begin() + s, members.begin() + std::min(members.size(), s + (size_t)G));
        for (int i : g) group_of[i] = (int)groups.size();
        groups.push_back(g);
        group_size_of.push_back(G);
      }
    }
  }

  // ---- key-ordered windows: ungrouped problems (k <= 4, N large enough, at most 16 columns;
  // per-point outputs under algorithm 1 only) that share an unpermuted Z column are searched in
  // that column's order ----
  std::vector<int> win_of(np, -1), win_key(np, -1);  // window set, key column (original index)
  P.wsets.clear();
  if (use_windows) {
    std::map<std::pair<const float*, int64_t>, int> by_key;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      if (group_of[i] >= 0 || p.k + 1 > 5 || p.dz < 1 || p.dx + p.dy + p.dz > kMaxDimsCompiled ||
          p.n < window_min_n(p.dx + p.dy + p.dz))
        continue;
      if ((p.eps_out || p.counts_out || p.local_out) && algorithm != 1) continue;
      int a_key = -1;
      for (int a = p.dx + p.dy; a < p.dx + p.dy + p.dz && a_key < 0; ++a)
        if (!p.perm[a]) a_key = a;
      if (a_key < 0) continue;
      const auto kk = std::make_pair(p.col[a_key], p.n);
      auto it = by_key.find(kk);
      if (it == by_key.end()) {
        it = by_key.emplace(kk, (int)P.wsets.size()).first;
        P.wsets.push_back(kk);
      }
      win_of[i] = it->second;
      win_key[i] = a_key;
    }
  }

  // ---- column pool: pack every column that is not already a padded device column ----
  // Grouped problems address all their columns through one pool, so they always pack; so do
  // window problems, in their set's key order.
  struct Key {
    const float* src;
    const int32_t* perm;
    int64_t n;
    int wset;
    bool operator==(const Key& o) const { return src == o.src && perm == o.perm && n == o.n && wset == o.wset; }
  };
  struct KeyHash {
    size_t operator()(const Key& k) const {
      return std::hash<const void*>()(k.src) * 31u ^ std::hash<const void*>()(k.perm) ^ (size_t)k.n ^
             ((size_t)(k.wset + 1) << 20);
    }
  };
  std::unordered_map<Key, int64_t, KeyHash> slot;
  std::vector<PackJob>& jobs = P.jobs;
  jobs.clear();
  int64_t pool_floats = 0;
  int max_pad = 0;
  std::vector<std::array<int64_t, kMaxDims>> col_off(np);
  for (int i = 0; i < np; ++i) {
    const Problem& p = probs[i];
    const int D = p.dx + p.dy + p.dz;
    const int64_t n_pad = round_up(p.n, kPad);
    max_pad = std::max<int>(max_pad, (int)n_pad);
    for (int a = 0; a < D; ++a) {
      if (p.padded[a] && !p.perm[a] && group_of[i] < 0 && win_of[i] < 0) {
        col_off[i][a] = -1;  // used in place
        continue;
      }
      Key key{p.col[a], p.perm[a], p.n, win_of[i]};
      auto it = slot.find(key);
      if (it == slot.end()) {
        it = slot.emplace(key, pool_floats).first;
        PackJob j;
        j.src = p.col[a];
        j.perm = p.perm[a];
        j.dst = reinterpret_cast<float*>(pool_floats);  // offset for now
        j.n = (int)p.n;
        j.n_pad = (int)n_pad;
        // window set index + 1 for now (the key order's address is known after the pool is reserved)
        j.order = win_of[i] >= 0 ? reinterpret_cast<const int32_t*>((intptr_t)(win_of[i] + 1)) : nullptr;
        jobs.push_back(j);
        pool_floats += n_pad;
      }
      col_off[i][a] = it->second;
    }
  }
  P.max_pad = max_pad;
  // ---- wide problems (16 < D <= 32, not grouped): searched as problems of kWideDims columns,
  // their Z filled up with a zero column of the pool (exact: see ksg_search_wide.hip).  The
  // column is zero in the N rows and +inf in the padding rows, like every column, so that the
  // padding never enters a count: one per distinct N. ----
  std::vector<char> wide(np, 0);
  std::vector<int64_t> zero_off(np, -1);
  bool any_wide = false;
  {
    std::map<int64_t, int64_t> zero_of_n;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      wide[i] = group_of[i] < 0 && p.dx + p.dy + p.dz > kMaxDimsCompiled;
      if (!wide[i]) continue;
      any_wide = true;
      auto it = zero_of_n.find(p.n);
      if (it == zero_of_n.end()) {
        it = zero_of_n.emplace(p.n, pool_floats).first;
        PackJob j;
        std::memset(&j, 0, sizeof j);
        j.src = nullptr;                                // zeros, +inf padding
        j.dst = reinterpret_cast<float*>(pool_floats);  // offset for now
        j.n = (int)p.n;
        j.n_pad = (int)round_up(p.n, kPad);
        jobs.push_back(j);
        pool_floats += j.n_pad;
      }
      zero_off[i] = it->second;
    }
  }
  // key orders of the window sets (int32, n_pad entries each) follow the packed columns
  P.wsigma_off.assign(P.wsets.size(), 0);
  for (size_t w = 0; w < P.wsets.size(); ++w) {
    P.wsigma_off[w] = pool_floats;
    pool_floats += round_up(P.wsets[w].second, kPad);
  }
  // Interleaved blocks of the groups follow the packed columns in the same pool.
  std::vector<int64_t> xi_off(groups.size()), yzi_off(groups.size()), sigma_off(groups.size());
  std::vector<int> write_yz(groups.size(), 0);
  {
    std::map<std::vector<int64_t>, std::pair<int64_t, int64_t>> yz_sets;  // block, key order
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const int i0 = groups[gi][0];
      const int64_t n_pad = round_up(probs[i0].n, kPad);
      xi_off[gi] = pool_floats;
      pool_floats += (int64_t)group_size_of[gi] * n_pad;
      std::vector<int64_t> key = {n_pad};
      for (int a = 1; a < 2 + probs[i0].dz; ++a) key.push_back(col_off[i0][a]);
      auto it = yz_sets.find(key);
      if (it == yz_sets.end()) {
        const int64_t block = pool_floats;
        pool_floats += (int64_t)(probs[i0].dz + 1) * n_pad;
        const int64_t order = pool_floats;  // int32 row indices, one per padded row
        pool_floats += n_pad;
        it = yz_sets.emplace(key, std::make_pair(block, order)).first;
        write_yz[gi] = 1;
      }
      yzi_off[gi] = it->second.first;
      sigma_off[gi] = it->second.second;
    }
  }
  if (!groups.empty() && pool_floats > (int64_t)UINT32_MAX)
    return fail(KSG_ENOMEM, "batch needs %lld pool floats, above the 2^32 addressable by groups",
                (long long)pool_floats);
  st = reserve(pool, sizeof(float) * std::max<int64_t>(pool_floats, 1), "column pool");
  if (st) return st;
  float* pool_base = static_cast<float*>(pool.ptr);
  P.pool_base = pool_base;
  for (PackJob& j : jobs) {
    j.dst = pool_base + reinterpret_cast<int64_t>(j.dst);
    if (j.order) j.order = reinterpret_cast<const int32_t*>(pool_base + P.wsigma_off[(intptr_t)j.order - 1]);
  }
  // in-place columns: checked for finite values through identity jobs over their first n rows
  P.inplace.clear();
  for (int i = 0; i < np; ++i) {
    const Problem& p = probs[i];
    for (int a = 0; a < p.dx + p.dy + p.dz; ++a)
      if (col_off[i][a] < 0)
        P.inplace.push_back(PackJob{p.col[a], nullptr, const_cast<float*>(p.col[a]), (int)p.n, (int)p.n, nullptr});
  }

  auto cost = [&](int i) { return brute_cost(probs[i]); };
  auto n_tiles_of = [&](int i) { return (int)((probs[i].n + kTileQ - 1) / kTileQ); };
  // tile heights of the brute-force launches (algorithm 1): by the launch's size in 256-query tiles
  {
    int64_t t_plain = 0, t_wide = 0;
    for (int i = 0; i < np; ++i) {
      if (group_of[i] >= 0 || win_of[i] >= 0) continue;
      (wide[i] ? t_wide : t_plain) += n_tiles_of(i);
    }
    P.tile_q_plain = algorithm == 1 ? brute_tile_q(t_plain) : kTileQ;
    P.tile_q_wide = brute_tile_q(t_wide);
  }

  // ---- per-problem descriptors (search of ungrouped problems + finalisation of all) ----
  std::vector<int> order;
  for (int i = 0; i < np; ++i) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<ProbDesc>& descs = P.descs;
  descs.assign(np, ProbDesc{});
  int part = 0;
  // Group partial slots first (contiguous per group), then ungrouped problems.
  std::vector<int> group_part(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    group_part[gi] = part;
    part += (int)groups[gi].size() * n_tiles_of(groups[gi][0]);
  }
  P.common_shape = -2;
  P.kp = 5;
  int wide_kp = 5;
  for (int r = 0; r < np; ++r) {
    const int i = order[r];
    const Problem& p = probs[i];
    ProbDesc& d = descs[r];
    std::memset(&d, 0, sizeof d);
    const bool swap = p.dx > p.dy;
    const int dx = swap ? p.dy : p.dx, dy = swap ? p.dx : p.dy;
    const int D = p.dx + p.dy + p.dz;
    for (int a = 0; a < D; ++a) {
      int src = a;
      if (swap) {
        if (a < dx) src = p.dx + a;          // canonical X = original Y
        else if (a < dx + dy) src = a - dx;  // canonical Y = original X
      }
      d.col[a] = col_off[i][src] < 0 ? p.col[src] : pool_base + col_off[i][src];
    }
    if (wide[i])
      for (int a = D; a < kWideDims; ++a) d.col[a] = pool_base + zero_off[i];
    d.n = (int)p.n;
    d.n_pad = (int)round_up(p.n, kPad);
    d.dx = dx;
    d.dy = dy;
    d.dz = wide[i] ? kWideDims - dx - dy : p.dz;
    d.k = p.k;
    d.n_tiles = n_tiles_of(i);
    if (group_of[i] < 0 && win_of[i] < 0) {  // brute-force launches: their own tile height
      const int tq = wide[i] ? P.tile_q_wide : P.tile_q_plain;
      d.n_tiles = (int)((p.n + tq - 1) / tq);
    }
    d.eps_out = p.eps_out;
    d.counts_out = p.counts_out;
    d.local_out = p.local_out;
    d.variant = shape_id(dx, dy, p.dz);
    d.out_index = p.out_index;
    d.swap_xy = swap ? 1 : 0;
    d.alg = algorithm;
    d.key_col = win_key[i];  // a Z column: its index is the same in the canonical order
    d.key_order =
        win_of[i] >= 0 ? reinterpret_cast<const int32_t*>(pool_base + P.wsigma_off[win_of[i]]) : nullptr;
    if (group_of[i] >= 0) {
      const int gi = group_of[i];
      const int g = (int)(std::find(groups[gi].begin(), groups[gi].end(), i) - groups[gi].begin());
      d.part_base = group_part[gi] + g * d.n_tiles;
    } else if (win_of[i] >= 0) {
      d.part_base = part;
      part += d.n_tiles;
    } else if (wide[i]) {
      d.part_base = part;
      part += d.n_tiles;
      wide_kp = std::max(wide_kp, kp_for(p.k));
    } else {
      d.part_base = part;
      part += d.n_tiles;
      P.kp = std::max(P.kp, kp_for(p.k));
      // generic shapes share a kernel when their column counts agree
      const int launch_shape = d.variant >= kGenericShape ? kGenericShape + D : d.variant;
      if (P.common_shape == -2) P.common_shape = launch_shape;
      else if (P.common_shape != launch_shape) P.common_shape = -1;
    }
  }
  P.parts = part;

  // ---- ungrouped work items (algorithm 2: one launch per column count, items in D order) ----
  std::vector<WorkItem>& items = P.items;
  items.clear();
  P.segments.clear();
  P.plain_cost = 0.0;
  if (algorithm == 2) {
    std::map<int, std::vector<Unit>> by_d;
    std::map<int, int> kp_of;
    for (int r = 0; r < np; ++r) {
      const Problem& p = probs[order[r]];
      if (win_of[order[r]] >= 0) continue;  // searched in key order below
      const int D = p.dx + p.dy + p.dz;
      by_d[D].push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
      kp_of[D] = std::max(kp_of[D], kp_for(p.k));
    }
    for (auto& kv : by_d) {
      std::vector<WorkItem> seg = order_items(kv.second);
      double c = 0.0;
      for (const Unit& u : kv.second) c += u.cost;
      P.segments.push_back(BatchPlan::Segment{kv.first, kp_of[kv.first], (int)items.size(), (int)seg.size(), c});
      items.insert(items.end(), seg.begin(), seg.end());
    }
  } else {
    std::vector<Unit> units;
    for (int r = 0; r < np; ++r)
      if (group_of[order[r]] < 0 && win_of[order[r]] < 0 && !wide[order[r]])
        units.push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    for (const Unit& u : units) P.plain_cost += u.cost;
    items = order_items(units);
  }
  // items before the window and wide segments (brute-force items, or the algorithm-2 segments)
  P.n_plain_items = (int)items.size();
  // window problems: one launch per column count, after the other ungrouped items
  P.wsegments.clear();
  {
    std::map<int, std::vector<Unit>> by_d;
    for (int r = 0; r < np; ++r) {
      const Problem& p = probs[order[r]];
      if (win_of[order[r]] >= 0) by_d[p.dx + p.dy + p.dz].push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    }
    for (auto& kv : by_d) {
      std::vector<WorkItem> seg = order_items(kv.second);
      double c = 0.0;
      for (const Unit& u : kv.second) c += u.cost;
      P.wsegments.push_back(BatchPlan::Segment{kv.first, 5, (int)items.size(), (int)seg.size(), c});
      items.insert(items.end(), seg.begin(), seg.end());
    }
  }
  // wide problems: one launch of the kernel compiled for kWideDims columns
  P.wide_seg = BatchPlan::Segment{kWideDims, wide_kp, (int)items.size(), 0, 0.0};
  if (any_wide) {
    std::vector<Unit> units;
    for (int r = 0; r < np; ++r)
      if (wide[order[r]]) units.push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    std::vector<WorkItem> seg = order_items(units);
    for (const Unit& u : units) P.wide_seg.cost += u.cost;
    P.wide_seg.count = (int)seg.size();
    items.insert(items.end(), seg.begin(), seg.end());
  }

  // ---- groups: descriptors, launch chunks, Y/Z count descriptors, work items ----
  // Groups of one (m, G, KP) class run as chunks of consecutive groups, each chunk three
  // launches: radius (eps to E), Y/Z counts (terms to T), X counts (partial sums).  A chunk's
  // E (FP32) and T (FP64) hold G x n_pad elements per group, at most chunk_elems in all.
  const int64_t chunk_elems = group_chunk_elems > 0 ? group_chunk_elems : kGroupChunkElems;
  std::vector<GroupDesc>& gdescs = P.gdescs;
  gdescs.assign(groups.size(), GroupDesc{});
  std::map<std::array<int, 3>, std::vector<int>> class_groups;  // in creation order
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Problem& p0 = probs[groups[gi][0]];
    GroupDesc& gd = gdescs[gi];
    std::memset(&gd, 0, sizeof gd);
    const int i0 = groups[gi][0];
    for (int g = 0; g < kGroupMax; ++g) {
      const int i = groups[gi][g < (int)groups[gi].size() ? g : 0];
      gd.x_off[g] = (uint32_t)col_off[i][0];
    }
    gd.y_off = (uint32_t)col_off[i0][1];
    for (int a = 0; a < p0.dz; ++a) gd.z_off[a] = (uint32_t)col_off[i0][2 + a];
    gd.xi_off = (uint32_t)xi_off[gi];
    gd.yzi_off = (uint32_t)yzi_off[gi];
    gd.write_yz = write_yz[gi];
    gd.sigma_off = (uint32_t)sigma_off[gi];
    gd.G = group_size_of[gi];
    gd.n = (int)p0.n;
    gd.n_pad = (int)round_up(p0.n, kPad);
    gd.k = p0.k;
    gd.m = p0.dz;
    gd.ng = (int)groups[gi].size();
    gd.n_tiles = n_tiles_of(i0);
    gd.part_base = group_part[gi];
    class_groups[{p0.dz, group_size_of[gi], p0.k + 1 <= 5 ? 5 : 9}].push_back((int)gi);
  }
  P.chunks.clear();
  P.ydescs.clear();
  P.yitems.clear();
  P.chunk_elems_max = 0;
  for (auto& kv : class_groups) {
    const std::vector<int>& gl = kv.second;
    size_t a = 0;
    while (a < gl.size()) {
      // the chunk: groups gl[a, b)
      int64_t elems = 0;
      size_t b = a;
      while (b < gl.size()) {
        const int64_t e = (int64_t)gdescs[gl[b]].G * gdescs[gl[b]].n_pad;
        if (b > a && elems + e > chunk_elems) break;
        gdescs[gl[b]].e_off = (uint32_t)elems;
        elems += e;
        ++b;
      }
      P.chunk_elems_max = std::max(P.chunk_elems_max, elems);
      BatchPlan::Chunk c;
      c.cls = kv.first;
      std::vector<Unit> units;
      for (size_t q = a; q < b; ++q)
        units.push_back(Unit{gl[q], gdescs[gl[q]].n_tiles, cost(groups[gl[q]][0]) * gdescs[gl[q]].ng});
      std::stable_sort(units.begin(), units.end(), [](const Unit& u, const Unit& v) { return u.cost > v.cost; });
      c.items = order_items(units);
      // runs of consecutive groups of one Y/Z set -> slot ranges of at most kYZSlots
      c.ydesc_off = P.ydescs.size();
      const size_t y_first = P.yitems.size();
      size_t r0 = a;
      while (r0 < b) {
        size_t r1 = r0 + 1;
        while (r1 < b && gdescs[gl[r1]].yzi_off == gdescs[gl[r0]].yzi_off) ++r1;
        const GroupDesc& f = gdescs[gl[r0]];
        int n_valid = 0;  // groups are filled in order, only the last of a set can be short
        for (size_t q = r0; q < r1; ++q) n_valid = (int)(q - r0) * f.G + gdescs[gl[q]].ng;
        for (int s0 = 0; s0 < n_valid; s0 += kYZSlots) {
          YZDesc y;
          std::memset(&y, 0, sizeof y);
          y.yzi_off = f.yzi_off;
          y.e_off = f.e_off;
          y.n = f.n;
          y.n_pad = f.n_pad;
          y.G = f.G;
          y.slot0 = s0;
          y.n_slots = std::min(kYZSlots, n_valid - s0);
          const int di = (int)P.ydescs.size();
          P.ydescs.push_back(y);
          // One work-group per query row, rows handed out XCD-aware: in every block of 32 items
          // (32 rows), work-group b takes row 4 (b % 8) + (b % 32) / 8, so the four consecutive
          // rows whose radii share a 128-byte line of E go to work-groups b, b+8, b+16, b+24,
          // which the dispatcher places on one XCD (one L2 fetch instead of four).  Each
          // descriptor's items are padded to a multiple of 32 with empty items.
          const int nb = (f.n + 31) / 32;
          for (int b = 0; b < nb * 32; ++b) {
            const int row = 32 * (b / 32) + 4 * (b % 8) + (b % 32) / 8;
            P.yitems.push_back(row < f.n ? WorkItem{di, row} : WorkItem{-1, 0});
          }
        }
        r0 = r1;
      }
      c.n_ydesc = P.ydescs.size() - c.ydesc_off;
      c.n_yitems = P.yitems.size() - y_first;
      P.chunks.push_back(std::move(c));
      a = b;
    }
  }
  if (!groups.empty()) {
    st = reserve(ebuf, sizeof(float) * P.chunk_elems_max, "group radii");
    if (!st) st = reserve(tbuf, sizeof(double) * P.chunk_elems_max, "group count terms");
    if (st) return st;
  }
  // item layout of the upload: [ungrouped items | every chunk's items | Y/Z items]
  P.n_gitems = 0;
  for (BatchPlan::Chunk& c : P.chunks) {
    c.item_off = items.size() + P.n_gitems;
    P.n_gitems += c.items.size();
  }
  {
    size_t off = items.size() + P.n_gitems;  // Y/Z items follow, chunk after chunk
    for (BatchPlan::Chunk& c : P.chunks) {
      c.yitem_off = off;
      off += c.n_yitems;
    }
  }
  st = reserve(partials, sizeof(double) * std::max(part, 1), "partial sums");
  if (st) return st;
  // work counted on the host for the timing record: brute-force problems
  P.brute_ops = 0.0;
  for (int i = 0; i < np; ++i)
    if (group_of[i] < 0 && win_of[i] < 0) P.brute_ops += algorithmic_ops(probs[i], 1);
  P.n_groups = (int64_t)groups.size();
  return KSG_OK;
}

// ============================================================== upload

size_t BatchPlan::desc_bytes() const {
  return sizeof(ProbDesc) * descs.size() + sizeof(GroupDesc) * gdescs.size() + sizeof(YZDesc) * ydescs.size();
}
size_t BatchPlan::item_count() const { return items.size() + n_gitems + yitems.size(); }

// Copies descriptors, items and pack jobs through the pinned staging block into the three
// device buffers (stream-ordered).
int ksg_ctx::upload_batch(const BatchPlan& P, void* d_desc, void* d_items, void* d_jobs) {
  const size_t sz_desc = sizeof(ProbDesc) * P.descs.size();
  const size_t sz_g = sizeof(GroupDesc) * P.gdescs.size();
  const size_t sz_y = sizeof(YZDesc) * P.ydescs.size();
  const size_t sz_items = sizeof(WorkItem) * P.item_count();
  const size_t sz_jobs = sizeof(PackJob) * P.jobs.size();
  int st = reserve_host(sz_desc + sz_g + sz_y + sz_items + sz_jobs + 64);
  if (st) return st;
  char* h = static_cast<char*>(staging);
  std::memcpy(h, P.descs.data(), sz_desc);
  if (sz_g) std::memcpy(h + sz_desc, P.gdescs.data(), sz_g);
  if (sz_y) std::memcpy(h + sz_desc + sz_g, P.ydescs.data(), sz_y);
  char* hi = h + sz_desc + sz_g + sz_y;
  WorkItem* hw = reinterpret_cast<WorkItem*>(hi);
  if (!P.items.empty()) std::memcpy(hw, P.items.data(), sizeof(WorkItem) * P.items.size());
  for (const BatchPlan::Chunk& c : P.chunks)
    std::memcpy(hw + c.item_off, c.items.data(), sizeof(WorkItem) * c.items.size());
  if (!P.yitems.empty())
    std::memcpy(hw + P.items.size() + P.n_gitems, P.yitems.data(), sizeof(WorkItem) * P.yitems.size());
  char* hj = hi + sz_items;
  if (sz_jobs) std::memcpy(hj, P.jobs.data(), sz_jobs);
  KSG_HIP(this, hipMemcpyAsync(d_desc, h, sz_desc + sz_g + sz_y, hipMemcpyHostToDevice, stream));
  if (sz_items) KSG_HIP(this, hipMemcpyAsync(d_items, hi, sz_items, hipMemcpyHostToDevice, stream));
  if (sz_jobs) KSG_HIP(this, hipMemcpyAsync(d_jobs, hj, sz_jobs, hipMemcpyHostToDevice, stream));
  KSG_HIP(this, hipEventRecord(staging_done, stream));
  staging_pending = true;
  return KSG_OK;
}

// ============================================================== launches

int ksg_ctx::enqueue_batch(const BatchPlan& P, const void* d_desc_v, const WorkItem* d_items, const PackJob* d_jobs,
                           double* d_out) {
  int st = KSG_OK;
  const ProbDesc* d_desc = static_cast<const ProbDesc*>(d_desc_v);
  const GroupDesc* d_gdesc =
      reinterpret_cast<const GroupDesc*>(static_cast<const char*>(d_desc_v) + sizeof(ProbDesc) * P.descs.size());
  const YZDesc* d_ydesc = reinterpret_cast<const YZDesc*>(reinterpret_cast<const char*>(d_gdesc) +
                                                          sizeof(GroupDesc) * P.gdescs.size());
  float* pool_base = P.pool_base;
  const double* d_htab = static_cast<const double*>(htab.ptr);
  double* d_part = static_cast<double*>(partials.ptr);

  // ---- pack, optional finite check ----
  if (check_finite) KSG_HIP(this, hipMemsetAsync(d_flag, 0, sizeof(int), stream));
  for (size_t w = 0; w < P.wsets.size(); ++w)  // key orders first: the pack step reads them
    KSG_HIP(this, launch_window_rank(P.wsets[w].first, (int)P.wsets[w].second, (int)round_up(P.wsets[w].second, kPad),
                                     reinterpret_cast<int32_t*>(pool_base + P.wsigma_off[w]), stream));
  if (!P.jobs.empty()) KSG_HIP(this, launch_pack(d_jobs, (int)P.jobs.size(), P.max_pad, d_flag, stream));
  if (check_finite) {
    std::vector<PackJob> all = P.jobs;
    all.insert(all.end(), P.inplace.begin(), P.inplace.end());
    st = check_columns_finite(all, P.max_pad);
    if (st) return st;
  }
  if (!P.gdescs.empty()) {
    KSG_HIP(this, launch_key_order(d_gdesc, (int)P.gdescs.size(), P.max_pad, pool_base, stream));
    KSG_HIP(this, launch_interleave(d_gdesc, (int)P.gdescs.size(), P.max_pad, pool_base, stream));
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    t0 = get_event();
    t1 = get_event();
    if (!t0 || !t1) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(t0, stream));
  }
  float* d_e = static_cast<float*>(ebuf.ptr);
  double* d_t = static_cast<double*>(tbuf.ptr);
  unsigned long long* d_w = timing ? d_work : nullptr;
  // In timing mode every launch is bracketed by its own pair of events (per-kernel times),
  // recorded on the stream the launch goes to.
  hipEvent_t span_a = nullptr;
  auto span_begin = [&](hipStream_t st_) -> int {
    if (!timing) return KSG_OK;
    span_a = get_event();
    if (!span_a) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(span_a, st_));
    return KSG_OK;
  };
  auto span_end = [&](int kind, hipStream_t st_) -> int {
    if (!timing) return KSG_OK;
    hipEvent_t b = get_event();
    if (!b) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(b, st_));
    spans.push_back(Span{span_a, b, kind});
    return KSG_OK;
  };

  // Single-problem launches (one per column count or shape; none of them reads another's
  // output) are spread over the auxiliary streams, longest first onto the least-loaded
  // stream, so that launches too small to fill the device run side by side.  Grouped chunks
  // stay on the context's stream.
  struct Launch {
    int kind;  // 0 brute-force items, 1 window segment, 2 algorithm-2 segment, 3 wide problems
    int seg;
    double cost;
  };
  std::vector<Launch> launches;
  if (algorithm == 2) {
    for (size_t g = 0; g < P.segments.size(); ++g) launches.push_back(Launch{2, (int)g, P.segments[g].cost});
  } else if (P.n_plain_items > 0) {
    launches.push_back(Launch{0, 0, P.plain_cost});
  }
  for (size_t g = 0; g < P.wsegments.size(); ++g) launches.push_back(Launch{1, (int)g, P.wsegments[g].cost});
  if (P.wide_seg.count > 0) launches.push_back(Launch{3, 0, P.wide_seg.cost});
  const bool fork = launches.size() + (P.chunks.empty() ? 0 : 1) > 1;
  std::vector<hipStream_t> launch_stream(launches.size(), stream);
  bool aux_used[ksg_ctx::kAuxStreams] = {false, false, false};
  if (fork) {
    if ((st = ensure_aux_streams())) return st;
    std::vector<int> by_cost(launches.size());
    for (size_t i = 0; i < launches.size(); ++i) by_cost[i] = (int)i;
    std::stable_sort(by_cost.begin(), by_cost.end(),
                     [&](int a, int b) { return launches[a].cost > launches[b].cost; });
    // candidate streams: the context's (only when it runs no grouped chunk) and the auxiliaries
    std::vector<std::pair<hipStream_t, double>> load;
    if (P.chunks.empty()) load.emplace_back(stream, 0.0);
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i) load.emplace_back(aux_streams[i], 0.0);
    for (int li : by_cost) {
      size_t best = 0;
      for (size_t j = 1; j < load.size(); ++j)
        if (load[j].second < load[best].second) best = j;
      load[best].second += launches[li].cost;
      launch_stream[li] = load[best].first;
      for (int i = 0; i < ksg_ctx::kAuxStreams; ++i)
        if (load[best].first == aux_streams[i]) aux_used[i] = true;
    }
    KSG_HIP(this, hipEventRecord(fork_ev, stream));
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i)
      if (aux_used[i]) KSG_HIP(this, hipStreamWaitEvent(aux_streams[i], fork_ev, 0));
  }
  // Every launch is enqueued by this lambda; whatever it returns, the auxiliary streams are
  // joined back before the function returns, so that later work on the context's stream (and
  // a buffer reallocation, which synchronises that stream) orders after them.
  auto enqueue_search = [&]() -> int {
    for (size_t li = 0; li < launches.size(); ++li) {
      const Launch& L = launches[li];
      const hipStream_t ls = launch_stream[li];
      if ((st = span_begin(ls))) return st;
      if (L.kind == 3) {
        KSG_HIP(this, launch_ksg_search(d_desc, d_items + P.wide_seg.off, P.wide_seg.count, d_htab, d_part,
                                        kGenericShape + kWideDims, P.wide_seg.kp, ls, P.tile_q_wide));
      } else if (L.kind == 2) {
        const BatchPlan::Segment& g = P.segments[L.seg];
        KSG_HIP(this, launch_ksg_alg2(d_desc, d_items + g.off, g.count, d_htab, d_part, g.D, g.kp, ls));
      } else if (L.kind == 1) {
        const BatchPlan::Segment& g = P.wsegments[L.seg];
        KSG_HIP(this, launch_ksg_window(d_desc, d_items + g.off, g.count, d_htab, d_part, g.D, algorithm, d_w, ls));
      } else {
        KSG_HIP(this, launch_ksg_search(d_desc, d_items, P.n_plain_items, d_htab, d_part, P.common_shape, P.kp, ls,
                                        P.tile_q_plain));
      }
      if ((st = span_end(3, ls))) return st;
    }
    for (const BatchPlan::Chunk& c : P.chunks) {
      const int m = c.cls[0], G = c.cls[1], kp_c = c.cls[2];
      if ((st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_group_radius(pool_base, d_gdesc, d_items + c.item_off, (int)c.items.size(), d_e, m, G,
                                            kp_c, d_w, stream));
      if ((st = span_end(0, stream)) || (st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_yzcount(pool_base, d_ydesc, d_items + c.yitem_off, (int)c.n_yitems, d_e, d_t, d_htab,
                                       m, d_w, stream));
      if ((st = span_end(1, stream)) || (st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_group_xcount(pool_base, d_gdesc, d_items + c.item_off, (int)c.items.size(), d_e, d_t,
                                            d_htab, d_part, m, G, d_w, stream));
      if ((st = span_end(2, stream))) return st;
    }
    return KSG_OK;
  };
  const int st_search = enqueue_search();
  if (fork) {
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i) {
      if (!aux_used[i]) continue;
      hipError_t e = hipEventRecord(join_ev[i], aux_streams[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, join_ev[i], 0);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(aux_streams[i]);
        if (!st_search) return hip_fail(e, "joining an auxiliary stream");
      }
    }
  }
  if (st_search) return st_search;
  if (timing) {
    KSG_HIP(this, hipEventRecord(t1, stream));
    timed.emplace_back(t0, t1);
    timed_ops += P.brute_ops;  // window and grouped problems are counted by their kernels
  }
  KSG_HIP(this, launch_finalize(d_desc, P.np, d_part, d_htab, d_out, stream));
  return KSG_OK;
}

// ============================================================== entry

int ksg_ctx::run_batch(const std::vector<Problem>& probs, double* d_out) {
  if (probs.empty()) return KSG_OK;
  TraceRange range("ksg batch");
  if (use_graph && !timing && !check_finite) return run_batch_graph(probs, d_out);
  BatchPlan P;
  int st;
  {
    TraceRange r("ksg batch plan");
    st = plan_batch(probs, P);
  }
  if (st) return st;
  st = reserve(desc, std::max<size_t>(P.desc_bytes(), 16), "descriptors");
  if (!st) st = reserve(this->items, std::max<size_t>(sizeof(WorkItem) * P.item_count(), 16), "work items");
  if (!st) st = reserve(this->jobs, std::max<size_t>(sizeof(PackJob) * P.jobs.size(), 16), "pack jobs");
  if (st) return st;
  st = upload_batch(P, desc.ptr, this->items.ptr, this->jobs.ptr);
  if (st) return st;
  {
    TraceRange r("ksg batch enqueue");
    st = enqueue_batch(P, desc.ptr, static_cast<const WorkItem*>(this->items.ptr),
                       static_cast<const PackJob*>(this->jobs.ptr), d_out);
  }
  if (st) return st;
  last_items = (int64_t)P.item_count();
  last_groups = P.n_groups;
  return KSG_OK;
}

// ---- graph cache ----

// Everything the plan and the launches depend on besides the work buffers' addresses (which
// the buffer generation covers): the options, the tuned group sizes, the output and every
// problem's sizes, columns, gathers and outputs.
static std::vector<uint64_t> batch_key(const ksg_ctx* c, const std::vector<Problem>& probs, const double* d_out) {
  std::vector<uint64_t> key;
  key.reserve(8 + probs.size() * 12);
  key.push_back((uint64_t)probs.size());
  key.push_back((uint64_t)(uintptr_t)d_out);
  key.push_back((uint64_t)(int64_t)c->group_size);
  key.push_back((uint64_t)c->algorithm);
  key.push_back((uint64_t)c->use_windows | ((uint64_t)c->windows_untuned << 1));
  key.push_back((uint64_t)c->group_chunk_elems);
  key.push_back((uint64_t)c->tile_q);
  key.push_back((uint64_t)c->tuned);
  for (int t = 0; t < 2; ++t)
    for (int m = 0; m < 15; ++m) key.push_back((uint64_t)c->tuned_g[t][m]);
  key.push_back((uint64_t)c->tuned_tq[0]);
  key.push_back((uint64_t)c->tuned_tq[1]);
  for (int D = 0; D <= kMaxDimsCompiled; ++D) key.push_back((uint64_t)(int64_t)c->tuned_win_n[D]);
  for (const Problem& p : probs) {
    key.push_back((uint64_t)p.n);
    key.push_back(((uint64_t)p.dx << 48) | ((uint64_t)p.dy << 32) | ((uint64_t)p.dz << 16) | (uint64_t)p.k);
    key.push_back((uint64_t)(int64_t)p.out_index);
    const int D = p.dx + p.dy + p.dz;
    for (int a = 0; a < D; ++a) {
      key.push_back((uint64_t)(uintptr_t)p.col[a]);
      key.push_back((uint64_t)(uintptr_t)p.perm[a] ^ (p.padded[a] ? 1ull : 0ull));
    }
    key.push_back((uint64_t)(uintptr_t)p.eps_out);
    key.push_back((uint64_t)(uintptr_t)p.counts_out);
    key.push_back((uint64_t)(uintptr_t)p.local_out);
  }
  return key;
}

static uint64_t hash_key(const std::vector<uint64_t>& key) {
  uint64_t h = 1469598103934665603ull;
  for (uint64_t v : key) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 1099511628211ull;
  }
  return h;
}

void ksg_ctx::drop_graph(GraphEntry& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (DevBuf* b : {&g.desc, &g.items, &g.jobs}) {
    if (b->ptr) (void)hipFree(b->ptr);
    mem_held -= b->cap;
  }
  g = GraphEntry{};
}

void ksg_ctx::clear_graphs() {
  if (graphs.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (GraphEntry& g : graphs) drop_graph(g);
  graphs.clear();
}

int ksg_ctx::run_batch_graph(const std::vector<Problem>& probs, double* d_out) {
  std::vector<uint64_t> key = batch_key(this, probs, d_out);
  const uint64_t h = hash_key(key);
  for (GraphEntry& g : graphs) {
    if (g.hash == h && g.gen == buf_gen && g.key == key) {
      g.last_use = ++graph_clock;
      TraceRange r("ksg batch graph replay");
      KSG_HIP(this, hipGraphLaunch(g.exec, stream));
      last_items = g.n_items;
      last_groups = g.n_groups;
      ++graph_replays;
      return KSG_OK;
    }
  }
  // plan (may grow the shared work buffers, which retires the graphs that use them)
  BatchPlan P;
  int st = plan_batch(probs, P);
  if (st) return st;
  // graphs captured before a work buffer was reallocated can never be replayed: free them now
  bool stale = false;
  for (const GraphEntry& g : graphs) stale |= g.gen != buf_gen;
  if (stale) {
    (void)hipStreamSynchronize(stream);
    for (size_t i = graphs.size(); i-- > 0;)
      if (graphs[i].gen != buf_gen) {
        drop_graph(graphs[i]);
        graphs.erase(graphs.begin() + i);
      }
  }
  if (graphs.size() >= kMaxGraphs) {  // evict the least recently used
    size_t lru = 0;
    for (size_t i = 1; i < graphs.size(); ++i)
      if (graphs[i].last_use < graphs[lru].last_use) lru = i;
    (void)hipStreamSynchronize(stream);
    drop_graph(graphs[lru]);
    graphs.erase(graphs.begin() + lru);
  }
  GraphEntry g;
  struct Guard {  // releases a half-built entry on every error path
    ksg_ctx* c;
    GraphEntry* g;
    ~Guard() {
      if (g) c->drop_graph(*g);
    }
  } guard{this, &g};
  st = reserve(g.desc, std::max<size_t>(P.desc_bytes(), 16), "graph descriptors");
  if (!st) st = reserve(g.items, std::max<size_t>(sizeof(WorkItem) * P.item_count(), 16), "graph work items");
  if (!st) st = reserve(g.jobs, std::max<size_t>(sizeof(PackJob) * P.jobs.size(), 16), "graph pack jobs");
  if (st) return st;
  st = upload_batch(P, g.desc.ptr, g.items.ptr, g.jobs.ptr);
  if (st) return st;
  if ((st = ensure_aux_streams())) return st;
  if (!capture_stream) KSG_HIP(this, hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking));
  // Capture on a stream of our own (the context's may be the null stream, which cannot be
  // captured); the graph is launched on the context's stream.
  const hipStream_t saved = stream;
  stream = capture_stream;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  int st_enq = KSG_OK;
  if (e == hipSuccess) {
    st_enq = enqueue_batch(P, g.desc.ptr, static_cast<const WorkItem*>(g.items.ptr),
                           static_cast<const PackJob*>(g.jobs.ptr), d_out);
    e = hipStreamEndCapture(stream, &graph);
  }
  stream = saved;
  if (st_enq) {
    if (graph) (void)hipGraphDestroy(graph);
    return st_enq;
  }
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(e, "capturing the batch");
  }
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "instantiating the batch graph");
  KSG_HIP(this, hipGraphLaunch(g.exec, stream));
  g.key = std::move(key);
  g.hash = h;
  g.gen = buf_gen;
  g.last_use = ++graph_clock;
  g.n_items = (int64_t)P.item_count();
  g.n_groups = P.n_groups;
  last_items = g.n_items;
  last_groups = g.n_groups;
  ++graph_captures;
  graphs.push_back(std::move(g));
  guard.g = nullptr;
  return KSG_OK;
}

// Algorithmic FP32 operations (the roofline's work count).
// Ungrouped problem: the brute-force count over ordered pairs, N(N-1)(4D+2) (radius: D sub,
// D-1 max, 1 compare; counts: D sub, D-1 max, 3 compares).
// Grouped problems are counted by the kernels themselves, over the work they executed.
// Radius and X count kernels, in units of 4 references x 64 lanes: the shared part once per
// pair for the whole group -- radius d^YZ (2m+1: m+1 sub, m max) and the skip test (1); X
// counts d^Z (2m-1) and the skip test (1), nothing when m = 0 -- and the per-problem part,
// radius 3 (sub, max, compare) and X counts 3 (sub, max, compare) per pair, for every problem
// whose step ran.  Y/Z count kernel, in operations: per visited reference d^Z and d^YZ
// (2m+1, or 1) and one binary-search compare per level per rank (two ranks, one when m = 0).
// Steps outside a wave's key window are not executed and not counted.
double ksg_ctx::algorithmic_ops(const Problem& p, int) {
  const double pairs = (double)p.n * (double)(p.n - 1);
  return pairs * (4.0 * (p.dx + p.dy + p.dz) + 2.0);
}
