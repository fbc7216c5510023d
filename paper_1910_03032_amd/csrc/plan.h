// Host-side preparation of an order-p mesh for the library (no HIP): validation of the
// element->DoF map, the encoded map the element kernels read, and the assembly plan
// (which DoFs the assembly kernel writes and where their element contributions are).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace sfem {

// Encoding of the library-owned element->DoF map entries (int32):
//   bits 0..29  global DoF
//   bit 30      "sole": the DoF belongs to this element only (written directly)
//   bit 31      essential DoF (entry is negative)
constexpr int32_t kDofMask = 0x3fffffff;
constexpr int32_t kSoleBit = 0x40000000;

// E-vector layout used for order p (see HostPlan): DoF-ordered up to p = 4, where the
// assembly kernel's share of the apply is largest; element-ordered above, where the
// element kernel's scattered entry writes and the position table cost more than the
// assembly saves.
constexpr bool evec_dof_ordered(int p) { return p <= 4; }

struct HostPlan {
  bool compact = true;         // E-vector holds the surface nodes only (S per element)
  int64_t epe = 0;             // E-vector entries per element (S or n^3)
  std::vector<int32_t> imap;   // [nelem][n^3] encoded map
  // Assembly list: the DoFs the assembly kernel writes (shared or essential), ascending,
  // with CSR offsets aoff: alist[i] has aoff[i+1] - aoff[i] contributions, in element
  // order (essential DoFs have none).  Two E-vector layouts:
  //   DoF-ordered (dof_ordered): the contributions of alist[i] occupy the E-vector
  //     entries [aoff[i], aoff[i+1]), so the assembly reads them contiguously; pos maps
  //     an element node to its entry: index e * epe + r, r the node's surface rank
  //     (compact) or local index (general), -1 for nodes without an entry;
  //   element-ordered: the element writes its node r to entry e * epe + r, and slots
  //     [aoff[i], aoff[i+1]) hold the entries of alist[i]'s contributions.
  bool dof_ordered = true;
  std::vector<int32_t> alist;  // [na]
  std::vector<int32_t> aoff;   // [na + 1]
  std::vector<int32_t> pos;    // DoF-ordered: [nelem * epe]
  std::vector<int32_t> slots;  // element-ordered: [aoff[na]]
  int64_t na = 0;
  int64_t nentries = 0;        // E-vector entries per member
};

// Rank of local node l (l = i + n (j + n k), n = p + 1) among the element's surface nodes:
// face k = 0, face k = p, then for each interior k the ring of the (i, j) square; -1 for
// an interior node.
int64_t surface_rank(int p, int64_t l);

// Validates the map (range, no DoF twice in an element, every DoF used) and builds the
// plan.  Returns 0, or a negative sfem_status with err describing the problem.
int build_host_plan(int p, int64_t nelem, const int32_t *dofs, int64_t ndof, const uint8_t *ess,
                    HostPlan &out, std::string &err, bool dof_ordered = true);

}  // namespace sfem
