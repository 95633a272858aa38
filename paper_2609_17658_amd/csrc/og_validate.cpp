// og_tree_validate: a host-side check of a built tree's invariants (the
// structure the paper's "Tree construction" describes: particles in curve
// order, the recursive 8-way cube hierarchy in first-child / sibling
// order, node mass and centre of mass from a bottom-up pass), plus the
// derived walk records.  Slow by design (everything is copied to the host
// and checked node by node); meant for tests, debugging and audits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "og_forest.h"

using namespace og;

namespace {

// OG_FAULT_CORRUPT=<field> changes one value of the host copy before the
// checks run, so that tests can see each check fire without touching the
// device: keys, perm, position, count, skip, parent, level, mass, com, record.
void corrupt_copy(const char *what, std::vector<uint64_t> &keys, std::vector<uint32_t> &perm,
                  std::vector<double4> &part, std::vector<Topo> &topo, std::vector<uint32_t> &skip,
                  std::vector<uint32_t> &parent, std::vector<Mom64> &mom, std::vector<WNode> &wn) {
  const size_t n = keys.size(), nn = topo.size();
  const std::string w = what;
  if (w == "keys" && n >= 2) {  // two particles out of curve order
    std::swap(keys[0], keys[n - 1]);
    std::swap(part[0], part[n - 1]);
  }
  if (w == "perm" && n >= 2) perm[1] = perm[0];
  if (w == "position" && n >= 1) part[n / 2].x += 0.25 * (std::fabs(part[n / 2].x) + 1.0);
  if (w == "count" && nn >= 1) topo[nn - 1].b += 1u;
  if (w == "skip" && nn >= 2) skip[0] = (uint32_t)nn - 1u;
  if (w == "parent" && nn >= 2) parent[nn - 1] = (uint32_t)nn - 1u;
  if (w == "level" && nn >= 2) topo[1].b += 1u << kCountBits;
  if (w == "mass" && nn >= 1) mom[0].m *= 1.0 + 1e-6;
  if (w == "com" && nn >= 1) mom[nn - 1].cx += 1.0;
  if (w == "record" && nn >= 1) wn[0].cf ^= 1u;
}

struct Checker {
  int rc = OG_OK;
  template <class... Args>
  bool bad(const char *fmt, Args... args) {
    if (rc == OG_OK) rc = fail(OG_ECORRUPT, fmt, args...);
    return false;
  }
};

uint32_t axis(uint64_t corner, int k) { return (uint32_t)((corner >> (21 * k)) & 0x1fffffull); }

// Cell of a coordinate on the level-21 grid, as the key kernel forms it.
uint32_t cell(double x, double lo, double scale) {
  const double v = (x - lo) * scale;
  if (!(v >= 0.0)) return 0xffffffffu;
  if (v >= 2097151.0) return 2097151u;
  return (uint32_t)v;
}

}  // namespace

extern "C" int og_tree_validate(const og_tree *tree) {
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  const Forest &F = tree->F;
  if (F.B != 1) return fail(OG_EINVAL, "not a single-box tree");
  hipError_t e = hipStreamSynchronize(F.stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  {
    const int st = const_cast<Forest &>(F).read_status(F.stream);
    if (st != OG_OK) return st;
  }
  uint32_t sc[8];
  if ((e = hipMemcpy(sc, F.A.scalars, sizeof(sc), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(scalars)");
  const uint32_t N = F.N, nn = sc[3];
  if (nn > F.node_cap) return fail(OG_ECORRUPT, "node count %u above the capacity %u", nn, F.node_cap);
  BoxDev bx;
  if ((e = hipMemcpy(&bx, F.A.boxes, sizeof(bx), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(box)");
  std::vector<uint64_t> keys(N);
  std::vector<uint32_t> perm(N), first(nn), skip(nn), parent(nn);
  std::vector<double4> part(N);
  std::vector<Topo> topo(nn);
  std::vector<Mom64> mom(nn);
  std::vector<Mom32> m32(nn);
  std::vector<WNode> wn(nn);
  std::vector<double> seps, semax, semin;
  const bool soft = F.A.seps != nullptr;
  if (soft) {
    seps.resize(N);
    semax.resize(nn);
    semin.resize(nn);
  }
  hipError_t first_err = hipSuccess;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (first_err == hipSuccess && bytes) first_err = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  cp(keys.data(), F.A.keys_a, 8ull * N);
  cp(perm.data(), F.A.perm, 4ull * N);
  cp(part.data(), F.A.part64, sizeof(double4) * N);
  cp(first.data(), F.A.first, 4ull * nn);
  cp(skip.data(), F.A.skip, 4ull * nn);
  cp(parent.data(), F.A.parent, 4ull * nn);
  cp(topo.data(), F.A.topo, sizeof(Topo) * nn);
  cp(mom.data(), F.A.mom64, sizeof(Mom64) * nn);
  cp(m32.data(), F.A.mom32, sizeof(Mom32) * nn);
  cp(wn.data(), F.A.wnode, sizeof(WNode) * nn);
  if (soft) {
    cp(seps.data(), F.A.seps, 8ull * N);
    cp(semax.data(), F.A.semax, 8ull * nn);
    cp(semin.data(), F.A.semin, 8ull * nn);
  }
  if (first_err != hipSuccess) return hip_fail(first_err, "hipMemcpy(tree arrays)");
  if (const char *c = std::getenv("OG_FAULT_CORRUPT")) corrupt_copy(c, keys, perm, part, topo, skip, parent, mom, wn);

  Checker ck;
  // particles: keys sorted, perm a permutation, each key the key of its position
  std::vector<uint8_t> seen(N, 0);
  for (uint32_t p = 0; p < N && ck.rc == OG_OK; ++p) {
    if (p > 0 && keys[p] < keys[p - 1]) ck.bad("keys not sorted at %u", p);
    if (perm[p] >= N || seen[perm[p]]) ck.bad("perm is not a permutation (position %u)", p);
    else seen[perm[p]] = 1;
    const double x[3] = {part[p].x, part[p].y, part[p].z};
    uint32_t c[3];
    for (int k = 0; k < 3; ++k) {
      c[k] = cell(x[k], bx.lo[k], bx.scale);
      if (bx.periodic && !(x[k] < bx.box)) ck.bad("particle %u lies outside the periodic box", p);
    }
    if (c[0] > 2097151u || c[1] > 2097151u || c[2] > 2097151u) ck.bad("particle %u lies below the root cube", p);
    else if ((bx.curve ? hilbert3(c[0], c[1], c[2]) : morton3(c[0], c[1], c[2])) != keys[p])
      ck.bad("key of particle %u does not match its position", p);
  }
  if (ck.rc != OG_OK) return ck.rc;
  if (N == 0) return nn == 0 ? OG_OK : fail(OG_ECORRUPT, "%u nodes for no particles", nn);

  // root
  if (nn == 0) return fail(OG_ECORRUPT, "no nodes");
  if ((topo[0].b >> kCountBits) != 0 || (topo[0].b & kCountMask) != N || first[0] != 0 || skip[0] != nn ||
      parent[0] != 0xffffffffu)
    return fail(OG_ECORRUPT, "root node is not (level 0, particles [0,%u), skip %u, no parent)", N, nn);

  const double tol = 1e-12;
  for (uint32_t r = 0; r < nn && ck.rc == OG_OK; ++r) {
    const Topo &t = topo[r];
    const int lev = (int)(t.b >> kCountBits);
    const uint32_t cnt = t.b & kCountMask, f = first[r];
    const bool leaf = (t.corner & kLeafBit) != 0;
    if (lev > kLevels) { ck.bad("node %u at level %d", r, lev); break; }
    if (cnt == 0 || (uint64_t)f + cnt > N) { ck.bad("node %u holds particles [%u,%u+%u) outside [0,%u)", r, f, f, cnt, N); break; }
    if (leaf != (cnt <= (uint32_t)bx.leaf_max || lev == kLevels))
      ck.bad("node %u (level %d, %u particles) is %s a leaf", r, lev, cnt, leaf ? "wrongly" : "not");
    const int sh = kLevels - lev;
    for (int k = 0; k < 3; ++k)
      if ((axis(t.corner, k) & ((1u << sh) - 1u)) != 0) ck.bad("node %u corner not aligned to level %d", r, lev);
    // the particles lie in the node's cube: their keys share its prefix
    const uint64_t pref = lev == 0 ? 0 : keys[f] >> (3 * sh);
    if (lev > 0 && (keys[f + cnt - 1] >> (3 * sh)) != pref) ck.bad("particles of node %u leave its cube", r);
    if (bx.curve == 0 && lev > 0 &&
        (keys[f] >> (3 * sh)) != (morton3(axis(t.corner, 0), axis(t.corner, 1), axis(t.corner, 2)) >> (3 * sh)))
      ck.bad("node %u corner does not match its particles' keys", r);
    if (bx.curve != 0) {
      uint32_t c[3];
      hilbert3_cell(keys[f], c);
      for (int k = 0; k < 3; ++k)
        if ((c[k] >> sh) != (axis(t.corner, k) >> sh)) ck.bad("node %u corner does not match its keys", r);
    }
    // cube centre and side, as the build forms them
    const double h = bx.L * 0x1p-21, half = std::ldexp(1.0, 20 - lev), side = std::ldexp(bx.L, -lev);
    double cen[3];
    for (int k = 0; k < 3; ++k) cen[k] = bx.lo[k] + ((double)axis(t.corner, k) + half) * h;
    // moments
    double M = 0.0, s[3] = {0.0, 0.0, 0.0}, amax = 0.0;
    double ehi = 0.0, elo = INFINITY;
    if (leaf) {
      if (skip[r] != r + 1) ck.bad("leaf %u has skip %u", r, skip[r]);
      if (t.a != f) ck.bad("leaf %u record points at particle %u, not %u", r, t.a, f);
      for (uint32_t j = f; j < f + cnt; ++j) {
        M += part[j].w;
        amax += std::fabs(part[j].w);
        s[0] += part[j].w * (part[j].x - cen[0]);
        s[1] += part[j].w * (part[j].y - cen[1]);
        s[2] += part[j].w * (part[j].z - cen[2]);
        if (soft) {
          ehi = std::max(ehi, seps[j]);
          elo = std::min(elo, seps[j]);
        }
      }
    } else {
      if (t.a != skip[r]) ck.bad("node %u record skip %u differs from skip %u", r, t.a, skip[r]);
      if (skip[r] <= r + 1 || skip[r] > nn) { ck.bad("node %u has skip %u", r, skip[r]); break; }
      // children: r+1, then along skip, tiling the node's particle range
      uint32_t next = f, kids = 0, octs = 0;
      for (uint32_t ch = r + 1; ch < skip[r]; ch = skip[ch]) {
        if (skip[ch] <= ch || skip[ch] > skip[r]) { ck.bad("child %u of node %u has skip %u", ch, r, skip[ch]); break; }
        const int cl = (int)(topo[ch].b >> kCountBits);
        if (parent[ch] != r) ck.bad("node %u has parent %u, not %u", ch, parent[ch], r);
        if (cl != lev + 1) ck.bad("child %u of node %u at level %d, not %d", ch, r, cl, lev + 1);
        if (first[ch] != next) ck.bad("child %u of node %u starts at particle %u, not %u", ch, r, first[ch], next);
        if (cl == lev + 1 && sh >= 1) {
          uint32_t oct = 0;
          for (int k = 0; k < 3; ++k) {
            if ((axis(topo[ch].corner, k) >> sh) != (axis(t.corner, k) >> sh))
              ck.bad("child %u lies outside the cube of node %u", ch, r);
            oct |= ((axis(topo[ch].corner, k) >> (sh - 1)) & 1u) << k;
          }
          if (octs & (1u << oct)) ck.bad("two children of node %u in one octant", r);
          octs |= 1u << oct;
        }
        next += topo[ch].b & kCountMask;
        ++kids;
        M += mom[ch].m;
        amax += std::fabs(mom[ch].m);
        s[0] += mom[ch].m * (mom[ch].cx - cen[0]);
        s[1] += mom[ch].m * (mom[ch].cy - cen[1]);
        s[2] += mom[ch].m * (mom[ch].cz - cen[2]);
        if (soft) {
          ehi = std::max(ehi, semax[ch]);
          elo = std::min(elo, semin[ch]);
        }
        if (ck.rc != OG_OK) break;
      }
      if (ck.rc == OG_OK && (kids < 1 || kids > 8)) ck.bad("node %u has %u children", r, kids);
      if (ck.rc == OG_OK && next != f + cnt) ck.bad("children of node %u hold particles up to %u, not %u", r, next, f + cnt);
    }
    if (ck.rc != OG_OK) break;
    if (!(std::fabs(mom[r].m - M) <= tol * amax)) ck.bad("mass of node %u is %.17g, its contents sum to %.17g", r, mom[r].m, M);
    if (M > 0.0) {
      const double com[3] = {mom[r].cx, mom[r].cy, mom[r].cz};
      for (int k = 0; k < 3; ++k) {
        // a particle's cell comes from one rounded product, so it may lie an
        // ulp or so of its coordinate outside the exact cube
        if (!(std::fabs(com[k] - cen[k]) <= 0.5 * side * (1.0 + tol) + 4e-15 * (std::fabs(cen[k]) + bx.L)))
          ck.bad("centre of mass of node %u lies outside its cube", r);
        const double want = cen[k] + s[k] / M;
        if (!(std::fabs(com[k] - want) <= 1e-9 * side + 4.0 * tol * std::fabs(cen[k])))
          ck.bad("centre of mass of node %u is not its contents' (axis %d: %.17g vs %.17g)", r, k, com[k], want);
      }
      if (std::fabs((double)m32[r].m - M) > 1e-6 * std::fabs(M)) ck.bad("FP32 mass of node %u", r);
      const double o[3] = {m32[r].ox, m32[r].oy, m32[r].oz};
      for (int k = 0; k < 3; ++k)
        if (!(std::fabs(o[k] - (com[k] - cen[k])) <= 1e-6 * side)) ck.bad("FP32 offset of node %u", r);
    }
    if (soft && (semax[r] != ehi || semin[r] != elo)) ck.bad("softening range of node %u", r);
    // walk record
    const WNode &w = wn[r];
    const int hc = 1 << sh;
    for (int k = 0; k < 3; ++k)
      if (w.c[k] != (int32_t)(0x4B000000u | (uint32_t)(2 * (int)axis(t.corner, k) + hc)))
        ck.bad("walk record of node %u: centre", r);
    if ((w.cf & kWCount) != cnt || ((w.cf & kWLeaf) != 0) != leaf || ((w.cf & kWBig) != 0) != (leaf && cnt > 8u))
      ck.bad("walk record of node %u: count or flags", r);
    if (leaf ? (w.a & kTagFirst) != f || (w.a & kTagLeaf) == 0 || ((w.a >> 27) & 7u) + 1u != std::min(cnt, 8u)
             : w.a != skip[r])
      ck.bad("walk record of node %u: link", r);
  }
  return ck.rc;
}
