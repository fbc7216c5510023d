// Host test of the mesh preparation and assembly plan (plan.cpp), compiled with g++.
// For each mesh the plan is replayed on the CPU with integer element contributions and
// compared with a direct scatter-add over the element->DoF map; the map encoding, the
// class structure and the error paths are checked too.  Prints FAIL lines on mismatch.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "plan.h"
#include "sfem.h"

using namespace sfem;

static int failures = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      std::printf("FAIL: " __VA_ARGS__);  \
      std::printf("\n");                  \
      ++failures;                         \
    }                                     \
  } while (0)

// ne^3 box, order p, lexicographic elements and DoFs (the workloads' numbering)
static void box(int ne, int p, std::vector<int32_t> &dofs, std::vector<uint8_t> &ess, int64_t &ndof) {
  const int n = p + 1, n1 = ne * p + 1;
  ndof = (int64_t)n1 * n1 * n1;
  dofs.assign((size_t)ne * ne * ne * n * n * n, 0);
  ess.assign((size_t)ndof, 0);
  for (int ez = 0; ez < ne; ++ez)
    for (int ey = 0; ey < ne; ++ey)
      for (int ex = 0; ex < ne; ++ex) {
        const int e = ex + ne * (ey + ne * ez);
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              const int gx = ex * p + i, gy = ey * p + j, gz = ez * p + k;
              const int g = gx + n1 * (gy + n1 * gz);
              dofs[(size_t)e * n * n * n + i + n * (j + n * k)] = g;
              if (gx == 0 || gy == 0 || gz == 0 || gx == n1 - 1 || gy == n1 - 1 || gz == n1 - 1)
                ess[(size_t)g] = 1;
            }
      }
}

// Replays the plan: y_plan[g] from E-vector values vs the direct scatter-add.
static void replay1(const char *name, int p, int64_t nelem, const std::vector<int32_t> &dofs,
                    const std::vector<uint8_t> &ess, int64_t ndof, bool expect_compact, bool dof_ordered) {
  HostPlan hp;
  std::string err;
  const int rc = build_host_plan(p, nelem, dofs.data(), ndof, ess.data(), hp, err, dof_ordered);
  CHECK(rc == 0, "%s: build failed: %s", name, err.c_str());
  if (rc != 0) return;
  CHECK(hp.compact == expect_compact, "%s: compact = %d", name, (int)hp.compact);
  const int64_t n3 = (int64_t)(p + 1) * (p + 1) * (p + 1);
  std::vector<int64_t> deg((size_t)ndof, 0);
  for (int32_t g : dofs) deg[(size_t)g]++;
  // encoded map
  for (int64_t k = 0; k < nelem * n3; ++k) {
    const int32_t g = dofs[(size_t)k], v = hp.imap[(size_t)k];
    CHECK((v & kDofMask) == g, "%s: map entry %lld", name, (long long)k);
    CHECK((v < 0) == (ess[(size_t)g] != 0), "%s: essential bit %lld", name, (long long)k);
    CHECK(((v & kSoleBit) != 0) == (!ess[(size_t)g] && deg[(size_t)g] == 1), "%s: sole bit %lld",
          name, (long long)k);
  }
  // integer element contributions: value of (e, l) = 1000 e + l + 1, written to the
  // node's E-vector entry (pos[e * epe + r] when DoF-ordered, e * epe + r otherwise);
  // every entry the assembly reads is written exactly once
  CHECK((int64_t)hp.aoff.size() == hp.na + 1 && hp.aoff[0] == 0, "%s: offsets", name);
  CHECK(hp.nentries == (dof_ordered ? hp.aoff[(size_t)hp.na] : nelem * hp.epe), "%s: entry count", name);
  CHECK((int64_t)(dof_ordered ? hp.pos.size() : hp.slots.size()) ==
            (dof_ordered ? nelem * hp.epe : hp.aoff[(size_t)hp.na]), "%s: table size", name);
  std::vector<int64_t> Y((size_t)hp.nentries, 0), direct((size_t)ndof, 0);
  std::vector<int> hits((size_t)hp.nentries, 0);
  std::vector<int64_t> owner((size_t)hp.nentries, -1);
  for (int64_t e = 0; e < nelem; ++e)
    for (int64_t l = 0; l < n3; ++l) {
      const int32_t g = dofs[(size_t)(e * n3 + l)];
      const int64_t v = 1000 * e + l + 1;
      direct[(size_t)g] += v;
      const int64_t r = hp.compact ? surface_rank(p, l) : l;
      const bool shared = !(ess[(size_t)g] || deg[(size_t)g] == 1);
      int64_t q = -1;
      if (dof_ordered) {
        q = r >= 0 ? hp.pos[(size_t)(e * hp.epe + r)] : -1;
        if (!shared) {
          CHECK(q < 0, "%s: node (%lld, %lld) of a sole/essential DoF has an entry", name, (long long)e,
                (long long)l);
          continue;
        }
      } else {
        if (!shared) continue;
        q = e * hp.epe + r;
      }
      CHECK(q >= 0 && q < hp.nentries, "%s: entry range", name);
      if (q < 0 || q >= hp.nentries) continue;
      Y[(size_t)q] = v;
      hits[(size_t)q]++;
      owner[(size_t)q] = e;
    }
  for (int64_t k = 0; k < hp.nentries; ++k)
    CHECK(hits[(size_t)k] <= 1, "%s: entry %lld written %d times", name, (long long)k, hits[(size_t)k]);
  std::vector<char> seen((size_t)ndof, 0);
  int64_t nslot_used = 0;
  for (int64_t i = 0; i < hp.na; ++i) {
    const int32_t g = hp.alist[(size_t)i];
    CHECK(!seen[(size_t)g], "%s: DoF %d listed twice", name, g);
    seen[(size_t)g] = 1;
    if (i > 0) CHECK(hp.alist[(size_t)i - 1] < g, "%s: list not ascending", name);
    const int64_t a = hp.aoff[(size_t)i], d = hp.aoff[(size_t)i + 1] - a;
    if (ess[(size_t)g]) {
      CHECK(d == 0, "%s: essential DoF %d has %lld entries", name, g, (long long)d);
      continue;
    }
    CHECK(d == deg[(size_t)g], "%s: DoF %d has %lld entries, degree %lld", name, g, (long long)d,
          (long long)deg[(size_t)g]);
    int64_t sum = 0, last = -1;
    for (int64_t k = 0; k < d; ++k) {
      const int64_t q = dof_ordered ? a + k : hp.slots[(size_t)(a + k)];
      CHECK(q >= 0 && q < hp.nentries && hits[(size_t)q] == 1, "%s: DoF %d reads an unwritten entry", name, g);
      if (q < 0 || q >= hp.nentries) continue;
      CHECK(owner[(size_t)q] > last, "%s: contributions not in element order (DoF %d)", name, g);
      last = owner[(size_t)q];
      sum += Y[(size_t)q];
    }
    nslot_used += d;
    CHECK(sum == direct[(size_t)g], "%s: DoF %d assembled %lld, direct %lld", name, g,
          (long long)sum, (long long)direct[(size_t)g]);
  }
  for (int64_t g = 0; g < ndof; ++g) {
    const bool assembled = ess[(size_t)g] || deg[(size_t)g] > 1;
    CHECK((seen[(size_t)g] != 0) == assembled, "%s: DoF %lld listed = %d", name, (long long)g,
          (int)seen[(size_t)g]);
  }
  std::printf("%s (%s): na %lld, contributions %lld, compact %d\n", name,
              dof_ordered ? "DoF-ordered" : "element-ordered", (long long)hp.na, (long long)nslot_used,
              (int)hp.compact);
}

static void replay(const char *name, int p, int64_t nelem, const std::vector<int32_t> &dofs,
                   const std::vector<uint8_t> &ess, int64_t ndof, bool expect_compact) {
  replay1(name, p, nelem, dofs, ess, ndof, expect_compact, true);
  replay1(name, p, nelem, dofs, ess, ndof, expect_compact, false);
}

int main() {
  std::vector<int32_t> dofs;
  std::vector<uint8_t> ess;
  int64_t ndof;
  for (int p = 1; p <= 4; ++p) {
    box(3, p, dofs, ess, ndof);
    char name[64];
    std::snprintf(name, sizeof name, "box 3^3 p=%d", p);
    replay(name, p, 27, dofs, ess, ndof, true);
  }
  // box without essential DoFs: boundary nodes of one element only become sole
  box(2, 2, dofs, ess, ndof);
  std::fill(ess.begin(), ess.end(), 0);
  replay("box 2^3 p=2 no ess", 2, 8, dofs, ess, ndof, true);
  // three p = 1 elements sharing node 0 (degree 3) and node 1 (degree 2); other nodes
  // private
  {
    std::vector<int32_t> d(24);
    int next = 2;
    for (int e = 0; e < 3; ++e)
      for (int l = 0; l < 8; ++l) d[(size_t)(e * 8 + l)] = (l == 0) ? 0 : (l == 1 && e < 2) ? 1 : next++;
    std::vector<uint8_t> es((size_t)next, 0);
    es[(size_t)next - 1] = 1;
    replay("3 x p=1 sharing a node", 1, 3, d, es, next, true);
  }
  // an element-interior node shared by two elements: general (non-compact) layout
  {
    box(2, 2, dofs, ess, ndof);
    const int center = 13;
    const int32_t d0 = dofs[(size_t)0 * 27 + center], d1 = dofs[(size_t)1 * 27 + center];
    dofs[(size_t)1 * 27 + center] = d0;
    const int32_t last = (int32_t)ndof - 1;
    for (auto &v : dofs)
      if (v == last) v = d1;
    ess[(size_t)d1] = ess[(size_t)last];
    replay("shared interior node", 2, 8, dofs, ess, ndof - 1, false);
  }
  // error paths
  {
    HostPlan hp;
    std::string err;
    box(1, 2, dofs, ess, ndof);
    std::vector<int32_t> bad = dofs;
    bad[5] = (int32_t)ndof;
    CHECK(build_host_plan(2, 1, bad.data(), ndof, ess.data(), hp, err) == SFEM_E_MESH, "out-of-range DoF");
    bad = dofs;
    bad[5] = bad[6];
    CHECK(build_host_plan(2, 1, bad.data(), ndof, ess.data(), hp, err) == SFEM_E_MESH, "repeated DoF");
    std::vector<uint8_t> es2(ess);
    es2.push_back(0);
    CHECK(build_host_plan(2, 1, dofs.data(), ndof + 1, es2.data(), hp, err) == SFEM_E_MESH, "unused DoF");
  }
  std::printf(failures ? "%d failures\n" : "all plan checks passed\n", failures);
  return failures ? 1 : 0;
}
