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
// windows, so its blocks have B = W_l * W_g unknowns.  Every line is factored and solved with
// its x1-blocks eliminated from both ends towards the middle block n/2.  Factors are stored
// line after line (g major, l minor), each line's n blocks contiguous, each block B*B
// row-major.
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

}  // namespace

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
  // the lines on no middle group (the sweep's shape A covers them; see sweep_variants.h)
  for (int g = 0; g < plan.Gz; ++g)
    for (int l = 0; l < plan.Gy; ++l)
      if (g != plan.zmid && l != plan.ymid)
        plan.maxB_front = std::max(plan.maxB_front, plan.line_B[(size_t)g * plan.Gy + l]);
  for (const GroupInfo& gi : plan.groups)
    if (gi.W > plan.maxW) plan.maxW = gi.W;
  plan.total_elems = off;
  return HELM_OK;
}
