// Host-side partition of the sweep axes and the factor layout.
//
// Along x3 (outer sweep) and x2 (inner sweep) the nodes 1..b form group 0, handled as one
// block (Sec. 3: the first b layers, in the boundary PML); the rest is cut into groups of
// d nodes, the last possibly shorter (Sec. 4.2: several layers per auxiliary problem).
// The auxiliary window of group g >= 1 adds p moving-PML nodes below the group (Sec. 4.2:
// the auxiliary PML may be thinner than b).
//
// Line problem (g, l) pairs x3-group g with x2-group l; its grid is x1 = 1..n times the two
// windows, so its blocks have B = W_l * W_g unknowns.  Factors are stored line after line in
// the order the forward sweeps consume them (g major, l minor), each line's n blocks
// contiguous, each block B*B row-major.
#include "common.h"

int build_plan(int n, int b, int p, int d, Plan& plan, std::string& msg) {
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
  plan = Plan();
  plan.n = n;
  plan.b = b;
  plan.p = p;
  plan.d = d;
  plan.groups.push_back(GroupInfo{1, b, 1, b});
  for (int k = b + 1; k <= n; k += d) {
    int last = k + d - 1 < n ? k + d - 1 : n;
    plan.groups.push_back(GroupInfo{k, last, k - p, last - (k - p) + 1});
  }
  plan.G = (int)plan.groups.size();
  plan.line_off.resize((size_t)plan.G * plan.G);
  plan.line_B.resize((size_t)plan.G * plan.G);
  long long off = 0;
  for (int g = 0; g < plan.G; ++g) {
    for (int l = 0; l < plan.G; ++l) {
      int B = plan.groups[g].W * plan.groups[l].W;
      plan.line_off[(size_t)g * plan.G + l] = off;
      plan.line_B[(size_t)g * plan.G + l] = B;
      off += (long long)n * B * B;
      if (B > plan.maxB) plan.maxB = B;
    }
    if (plan.groups[g].W > plan.maxW) plan.maxW = plan.groups[g].W;
  }
  plan.total_elems = off;
  return HELM_OK;
}
