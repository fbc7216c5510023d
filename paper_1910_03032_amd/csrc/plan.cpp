// Host-side mesh preparation and assembly plan (see plan.h).
#include "plan.h"

#include "sfem.h"

namespace sfem {

namespace {
int set_err(std::string &err, int code, const std::string &msg) {
  err = msg;
  return code;
}
}  // namespace

int64_t surface_rank(int p, int64_t l) {
  const int64_t n = p + 1;
  const int64_t i = l % n, j = (l / n) % n, k = l / (n * n);
  if (p == 1) return l;
  if (k == 0) return i + n * j;
  if (k == p) return n * n + i + n * j;
  const int64_t base = 2 * n * n + (k - 1) * 4 * p;
  if (j == 0) return base + i;
  if (j == p) return base + n + i;
  if (i == 0 || i == p) return base + 2 * n + 2 * (j - 1) + (i == 0 ? 0 : 1);
  return -1;
}

int build_host_plan(int p, int64_t nelem, const int32_t *dofs_ptr, int64_t ndof,
                    const uint8_t *ess_ptr, HostPlan &out, std::string &err, bool dof_ordered) {
  out = HostPlan{};
  out.dof_ordered = dof_ordered;
  const int n = p + 1;
  const int64_t n3 = (int64_t)n * n * n;
  auto dofs = [&](size_t k) { return dofs_ptr[k]; };
  std::vector<uint8_t> ess(ess_ptr, ess_ptr + ndof);
  // ---- validate the map: range, no repeated DoF inside an element, every DoF used
  std::vector<int64_t> deg((size_t)ndof + 1, 0);
  {
    std::vector<int64_t> stamp((size_t)ndof, -1);
    for (int64_t e = 0; e < nelem; ++e) {
      for (int64_t l = 0; l < n3; ++l) {
        const int32_t gd = dofs((size_t)(e * n3 + l));
        if (gd < 0 || gd >= ndof)
          return set_err(err, SFEM_E_MESH, "elem_dofs[" + std::to_string(e) + "][" + std::to_string(l) +
                                          "] = " + std::to_string(gd) + " is outside [0, ndof)");
        if (stamp[gd] == e)
          return set_err(err, SFEM_E_MESH, "element " + std::to_string(e) + " references DoF " +
                                          std::to_string(gd) + " twice");
        stamp[gd] = e;
        deg[gd]++;
      }
    }
    for (int64_t gd = 0; gd < ndof; ++gd)
      if (deg[gd] == 0)
        return set_err(err, SFEM_E_MESH, "DoF " + std::to_string(gd) + " belongs to no element");
  }
  // ---- a DoF referenced by one element only is written directly by that element
  // ("sole"); the others, and the essential DoFs, are written by the assembly kernel
  // from the E-vector.  Compact position table: indexed by the element's surface nodes
  // only, valid when every element-interior local node is sole or essential.
  const int64_t S = (p == 1) ? 8 : (int64_t)(2 * n * n + (n - 2) * 4 * p);
  bool compact = true;
  for (int64_t e = 0; e < nelem && compact; ++e)
    for (int64_t l = 0; l < n3; ++l) {
      const int32_t gd = dofs((size_t)(e * n3 + l));
      if (surface_rank(p, l) < 0 && !(deg[gd] == 1 || ess[gd])) {
        compact = false;
        break;
      }
    }
  const int64_t epe = compact ? S : n3;
  out.compact = compact;
  out.epe = epe;
  if (nelem * epe >= (int64_t)INT32_MAX) return set_err(err, SFEM_E_ARG, "mesh too large");
  std::vector<int32_t> &imap = out.imap;
  imap.assign((size_t)(nelem * n3), 0);
  for (int64_t e = 0; e < nelem; ++e)
    for (int64_t l = 0; l < n3; ++l) {
      const int32_t gd = dofs((size_t)(e * n3 + l));
      int32_t v = gd;
      if (ess[gd])
        v |= (int32_t)0x80000000u;
      else if (deg[gd] == 1)
        v |= kSoleBit;
      imap[(size_t)(e * n3 + l)] = v;
    }
  // assembled DoFs (shared or essential), ascending; the E-vector entries of their
  // contributions are contiguous per DoF, in element order
  std::vector<int32_t> apos((size_t)ndof, -1);
  std::vector<int32_t> &alist = out.alist;
  for (int64_t gd = 0; gd < ndof; ++gd)
    if (ess[gd] || deg[gd] > 1) {
      apos[gd] = (int32_t)alist.size();
      alist.push_back((int32_t)gd);
    }
  const int64_t na = (int64_t)alist.size();
  out.na = na;
  std::vector<int32_t> &aoff = out.aoff;
  aoff.assign((size_t)na + 1, 0);
  for (int64_t gd = 0; gd < ndof; ++gd)
    if (apos[gd] >= 0 && !ess[gd]) aoff[(size_t)apos[gd] + 1] = (int32_t)deg[gd];
  for (int64_t i = 0; i < na; ++i) aoff[(size_t)i + 1] += aoff[(size_t)i];
  std::vector<int32_t> next(aoff.begin(), aoff.end() - 1);
  if (dof_ordered) {
    out.nentries = aoff[(size_t)na];
    std::vector<int32_t> &pos = out.pos;
    pos.assign((size_t)(nelem * epe), -1);
    for (int64_t e = 0; e < nelem; ++e)
      for (int64_t l = 0; l < n3; ++l) {
        const int32_t gd = dofs((size_t)(e * n3 + l));
        if (ess[gd] || deg[gd] == 1) continue;
        pos[(size_t)(e * epe + (compact ? surface_rank(p, l) : l))] = next[(size_t)apos[gd]]++;
      }
  } else {
    out.nentries = nelem * epe;
    std::vector<int32_t> &slots = out.slots;
    slots.assign((size_t)aoff[(size_t)na], -1);
    for (int64_t e = 0; e < nelem; ++e)
      for (int64_t l = 0; l < n3; ++l) {
        const int32_t gd = dofs((size_t)(e * n3 + l));
        if (ess[gd] || deg[gd] == 1) continue;
        slots[(size_t)next[(size_t)apos[gd]]++] = (int32_t)(e * epe + (compact ? surface_rank(p, l) : l));
      }
  }
  return 0;
}

}  // namespace sfem
