// Host-side partition of the sweep axes and the factor layout.
//
// An axis swept from one face: the nodes 1..b form group 0, handled as one block (Sec. 3: the
// first b layers, in the boundary PML); the rest is cut into groups of d nodes, the last
// possibly shorter (Sec. 4.2: several layers per auxiliary problem).  The auxiliary window of
// group g >= 1 adds p moving-PML nodes below the group (Sec. 4.2: the auxiliary PML may be
// thinner than b).
//
// An axis swept from both faces (Sec. 4.2 note 3, the configuration of Sec. 5): the b layers
// at each face form the first and the last group, the interior is cut into groups of d;
// groups below the middle group (index G/2) are padded with p moving-PML nodes below, groups
// above it with p nodes above, the middle group on both sides; the first and last groups are
// not padded.  x3 (outer sweep) and x2 (inner sweep) choose independently.
//
// Line problem (g, l) pairs x3-group g with x2-group l; its grid is x1 = 1..n times the two
// windows, so its blocks have B = W_l * W_g unknowns.  The sweep solves the lines of a launch
// with two chains per workgroup when every block of the launch fits (B <= 64), else with one
// chain; a line's factors are in the elimination order its launches use (two-sided, or x1
// order).  Factors are stored line after line
// (g major, l minor), each line's n blocks contiguous, each block B*B row-major.
#include <algorithm>

#include "common.h"

namespace {

std::vector<GroupInfo> one_front_groups(int n, int b, int p, int d) {
  std::vector<GroupInfo> gs;
  gs.push_back(GroupInfo{1, b, 1, b});
  for (int k = b + 1; k <= n; k += d) {
    const int last = k + d - 1 < n ? k + d - 1 : n;
    gs.push_back(GroupInfo{k, last, k - p, last - (k - p) + 1});
  }
  return gs;
}

std::vector<GroupInfo> two_front_groups(int n, int b, int p, int d) {
  std::vector<std::pair<int, int>> cut;
  cut.push_back({1, b});
  for (int k = b + 1; k <= n - b; k += d) cut.push_back({k, k + d - 1 < n - b ? k + d - 1 : n - b});
  cut.push_back({n - b + 1, n});
  const int G = (int)cut.size(), mid = G / 2;
  std::vector<GroupInfo> gs;
  for (int g = 0; g < G; ++g) {
    const int a = cut[g].first, e = cut[g].second;
    int w0 = a, w1 = e;
    if (g > 0 && g < G - 1) {
      if (g <= mid) w0 = a - p;
      if (g >= mid) w1 = e + p;
    }
    gs.push_back(GroupInfo{a, e, w0, w1 - w0 + 1});
  }
  return gs;
}

// calls fn(launch, lines) for every launch of one sweep, in order (chains and maxB unset).
//   One inner front: one launch per outer pass, every workgroup sweeping its slabs and, in
//   each, all lines (pass 0 with one front; passes 1, 2, 3 with two).
//   Two inner fronts: per slab step of each outer pass, three launches: both inner fronts
//   forward (two workgroups per outer front), the middle line, both inner fronts backward;
//   the launch boundaries order them.
// The timed (dominant) launches are those over the front slabs' lines off the middle
// x2-group.
template <typename F> void for_each_launch(const Plan& P, F fn) {
  struct Outer {
    int pass, nfront;
  };
  const std::vector<Outer> outer =
      P.fronts == 1 ? std::vector<Outer>{{0, 1}} : std::vector<Outer>{{1, 2}, {2, 1}, {3, 2}};
  std::vector<int> lines;
  for (const Outer& o : outer) {
    const bool mid_slab = o.pass == 2;
    if (P.fronts_inner == 1) {
      lines.clear();
      for (int g = 0; g < P.Gz; ++g)
        if ((P.fronts == 2 && g == P.zmid) == mid_slab)
          for (int l = 0; l < P.Gy; ++l) lines.push_back(g * P.Gy + l);
      if (!lines.empty()) fn(SweepLaunch{o.pass, o.nfront, 0, 1 << 30, 0, 1, 0, 0, !mid_slab}, lines);
      continue;
    }
    int steps = 0;
    for (int fr = 0; fr < o.nfront; ++fr) steps = std::max(steps, sweep_count(o.pass, P.Gz, P.zmid, fr));
    for (int si = 0; si < steps; ++si) {
      for (int ip : {1, 2, 3}) {
        const int ninner = ip == 2 ? 1 : 2;
        lines.clear();
        for (int fr = 0; fr < o.nfront; ++fr) {
          if (si >= sweep_count(o.pass, P.Gz, P.zmid, fr)) continue;
          const int g = sweep_at(o.pass, P.Gz, P.zmid, fr, si).x;
          for (int inf = 0; inf < ninner; ++inf)
            for (int k = 0; k < sweep_count(ip, P.Gy, P.ymid, inf); ++k)
              lines.push_back(g * P.Gy + sweep_at(ip, P.Gy, P.ymid, inf, k).x);
        }
        if (!lines.empty())
          fn(SweepLaunch{o.pass, o.nfront, si, si + 1, ip, ninner, 0, 0, !mid_slab && ip != 2}, lines);
      }
    }
  }
}

}  // namespace

std::vector<SweepLaunch> sweep_schedule(const Plan& P) {
  std::vector<SweepLaunch> out;
  for_each_launch(P, [&](SweepLaunch L, const std::vector<int>& lines) {
    for (int line : lines) L.maxB = std::max(L.maxB, P.line_B[line]);
    L.chains = P.one[lines[0]] ? 1 : 2;   // the lines of a launch agree (build_plan)
    out.push_back(L);
  });
  return out;
}

int build_plan(int n, int b, int p, int d, int fronts, int fronts_inner, int prec, Plan& plan,
               std::string& msg) {
  if (b < 1 || n < 2 * b + 1) {
    msg = "need b >= 1 and n >= 2b+1";
    return HELM_EINVAL;
  }
  if (p < 0 || p > b) {
    msg = "need 0 <= p <= b (the moving PML must stay inside the domain)";
    return HELM_EINVAL;
  }
  if (d < 1) {
    msg = "need slab_layers >= 1";
    return HELM_EINVAL;
  }
  if (fronts != 1 && fronts != 2) {
    msg = "fronts must be 1 or 2";
    return HELM_EINVAL;
  }
  if (fronts_inner != 1 && fronts_inner != 2) {
    msg = "fronts_inner must be 1 or 2";
    return HELM_EINVAL;
  }
  plan = Plan();
  plan.n = n;
  plan.b = b;
  plan.p = p;
  plan.d = d;
  plan.fronts = fronts;
  plan.fronts_inner = fronts_inner;
  const std::vector<GroupInfo> zs = fronts == 2 ? two_front_groups(n, b, p, d) : one_front_groups(n, b, p, d);
  const std::vector<GroupInfo> ys =
      fronts_inner == 2 ? two_front_groups(n, b, p, d) : one_front_groups(n, b, p, d);
  if (fronts == 2) plan.zmid = (int)zs.size() / 2;
  if (fronts_inner == 2) plan.ymid = (int)ys.size() / 2;
  plan.Gz = (int)zs.size();
  plan.Gy = (int)ys.size();
  plan.groups = zs;
  plan.groups.insert(plan.groups.end(), ys.begin(), ys.end());
  plan.line_off.resize((size_t)plan.Gz * plan.Gy);
  plan.line_B.resize((size_t)plan.Gz * plan.Gy);
  long long off = 0;
  for (int g = 0; g < plan.Gz; ++g) {
    for (int l = 0; l < plan.Gy; ++l) {
      const int B = plan.zg(g).W * plan.yg(l).W;
      plan.line_off[(size_t)g * plan.Gy + l] = off;
      plan.line_B[(size_t)g * plan.Gy + l] = B;
      off += (long long)n * B * B;
      if (B > plan.maxB) plan.maxB = B;
    }
  }
  // chain counts: a launch holding a block above two_cap is solved by one chain, and so is
  // every line in it; a line sits in a forward and a backward launch whose other lines may
  // differ, so the marking repeats until every launch agrees
  plan.two_cap = prec == HELM_C64 ? kTwoChainMaxB64 : kTwoChainMaxB128;
  plan.one.assign((size_t)plan.Gz * plan.Gy, 0);
  for (bool changed = true; changed;) {
    changed = false;
    for_each_launch(plan, [&](const SweepLaunch&, const std::vector<int>& lines) {
      bool one = false;
      for (int line : lines) one = one || plan.one[line] || plan.line_B[line] > plan.two_cap;
      if (!one) return;
      for (int line : lines)
        if (!plan.one[line]) {
          plan.one[line] = 1;
          changed = true;
        }
    });
  }
  for (int g = 0; g < plan.Gz; ++g) {
    for (int l = 0; l < plan.Gy; ++l) {
      const int B = plan.line_B[(size_t)g * plan.Gy + l];
      if (plan.one_chain(g, l)) {
        if (B > plan.maxB_mid) plan.maxB_mid = B;
      } else if (B > plan.maxB_front) {
        plan.maxB_front = B;
      }
    }
  }
  for (const GroupInfo& gi : plan.groups)
    if (gi.W > plan.maxW) plan.maxW = gi.W;
  plan.total_elems = off;
  return HELM_OK;
}
