// Host-side plan and stream header of libdls.
//
// The stream keeps the shape of the paper's file (Sec. 2.7.2): a fixed,
// addressable header recording where each batch of 1000 patches starts and
// how long it is, followed by the packed, independently decodable batches.
//
// Header, little-endian:
//   char[4] "DLS1"; u32 version = 2; u32 header_bytes; u32 flags (bit0 adaptive,
//   bit1 L2 mode: bounds are NRMSE targets, batches hold ranks, steps, qV, qA
//   and raw values; bit2 global-basis mode: window 1, the batch table ends
//   with one basis batch per variable)
//   i32 ndim, nvars, dtype (0 f32, 1 f64), r_max
//   i64 nx, ny, nz, nt
//   i32 px, py, pz, pmin, window, batch_blocks (= 1000)
//   u64 nblocks; u32 nbatches; u32 extra (global-basis mode: basis kind)
//   f64 eps[nvars]
//   per variable: u32 nbits, ceil(nbits / 8) bytes of split bits, LSB first
//   per batch: u64 offset (from the end of the header), u64 compressed size,
//              u64 uncompressed size
#include <algorithm>
#include <cstring>

#include "../../include/dls.h"
#include "dls_internal.h"

namespace dls {

namespace {
constexpr uint32_t kVersion = 2;
constexpr size_t kFixed = 104;

template <typename T>
void put(std::vector<uint8_t>& out, T v) {
  uint8_t b[sizeof(T)];
  std::memcpy(b, &v, sizeof(T));
  out.insert(out.end(), b, b + sizeof(T));
}

template <typename T>
T get(const uint8_t* p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

std::vector<Leaf> uniform_leaves(const Problem& p) {
  std::vector<Leaf> out;
  for (int64_t z0 = 0; z0 < p.nz; z0 += p.pz)
    for (int64_t y0 = 0; y0 < p.ny; y0 += p.py)
      for (int64_t x0 = 0; x0 < p.nx; x0 += p.px)
        out.push_back(Leaf{int32_t(x0), int32_t(y0), int32_t(z0),
                           int32_t(std::min<int64_t>(p.px, p.nx - x0)),
                           int32_t(std::min<int64_t>(p.py, p.ny - y0)),
                           int32_t(std::min<int64_t>(p.pz, p.nz - z0))});
  return out;
}

// Depth-first rebuild of the quadtree / octree from split bits: a node of
// nominal edge e > pmin consumes one bit; 1 = split into the half-edge
// children whose origin lies in the domain, visited in (z, y, x) order.
// Leaves are returned sorted by (z0, y0, x0).
std::vector<Leaf> leaves_from_bits(const Problem& p, const std::vector<uint8_t>& bits, bool* ok) {
  std::vector<Leaf> out;
  size_t pos = 0;
  *ok = true;
  const bool is3d = p.nz > 1;
  struct Node { int64_t x0, y0, z0; int e; };
  std::vector<Node> stack;
  auto visit_root = [&](int64_t x0, int64_t y0, int64_t z0) {
    stack.push_back(Node{x0, y0, z0, p.px});
    while (!stack.empty() && *ok) {
      Node n = stack.back();
      stack.pop_back();
      if (n.e > p.pmin) {
        if (pos >= bits.size()) { *ok = false; return; }
        bool split = bits[pos++] != 0;
        if (split) {
          int h = n.e / 2;
          // push in reverse so children pop in (z, y, x) order
          std::vector<Node> kids;
          for (int dz = 0; dz < (is3d ? 2 : 1); ++dz)
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx) {
                int64_t cx = n.x0 + dx * h, cy = n.y0 + dy * h, cz = n.z0 + dz * h;
                if (cx < p.nx && cy < p.ny && cz < p.nz) kids.push_back(Node{cx, cy, cz, h});
              }
          for (auto it = kids.rbegin(); it != kids.rend(); ++it) stack.push_back(*it);
          continue;
        }
      }
      out.push_back(Leaf{int32_t(n.x0), int32_t(n.y0), int32_t(n.z0),
                         int32_t(std::min<int64_t>(n.e, p.nx - n.x0)),
                         int32_t(std::min<int64_t>(n.e, p.ny - n.y0)),
                         int32_t(is3d ? std::min<int64_t>(n.e, p.nz - n.z0) : 1)});
    }
  };
  const int e0 = p.px;
  for (int64_t z0 = 0; z0 < p.nz; z0 += (is3d ? e0 : 1))
    for (int64_t y0 = 0; y0 < p.ny; y0 += e0)
      for (int64_t x0 = 0; x0 < p.nx; x0 += e0) {
        visit_root(x0, y0, z0);
        if (!*ok) return {};
      }
  if (pos != bits.size()) *ok = false;
  std::stable_sort(out.begin(), out.end(), [](const Leaf& a, const Leaf& b) {
    if (a.z0 != b.z0) return a.z0 < b.z0;
    if (a.y0 != b.y0) return a.y0 < b.y0;
    return a.x0 < b.x0;
  });
  return out;
}

void build_blocks(const Problem& p, Plan& plan, int slice_points) {
  plan.blocks.clear();
  plan.items.clear();
  plan.item_start.clear();
  plan.code_off.clear();
  size_t nleaves = 0;
  for (int v = 0; v < p.nvars; ++v) nleaves += plan.leaves[v].size();
  const size_t nb_est = nleaves * size_t((p.nt + p.window - 1) / p.window);
  plan.blocks.reserve(nb_est);
  plan.code_off.reserve(nb_est);
  plan.item_start.reserve(nb_est + 1);
  plan.items.reserve(nb_est);
  int64_t off = 0;
  for (int v = 0; v < p.nvars; ++v) {
    for (int64_t t0 = 0; t0 < p.nt; t0 += p.window) {
      int w = int(std::min<int64_t>(p.window, p.nt - t0));
      for (const Leaf& L : plan.leaves[v]) {
        BlockDesc d;
        d.x0 = L.x0; d.y0 = L.y0; d.z0 = L.z0; d.t0 = int32_t(t0);
        d.ext = L.ex | (L.ey << 8) | (L.ez << 16) | (w << 24);
        d.var = v;
        d.m = L.ex * L.ey * L.ez;
        d.vec = (L.ex % 4 == 0 && L.x0 % 4 == 0 && p.nx % 4 == 0) ? 1 : 0;
        plan.item_start.push_back(int32_t(plan.items.size()));
        int rows = L.ey * L.ez;
        int rows_per = std::max(1, slice_points / L.ex);
        for (int r0 = 0; r0 < rows; r0 += rows_per) {
          int nr = std::min(rows_per, rows - r0);
          plan.items.push_back(Item{int32_t(plan.blocks.size()), r0 * L.ex, nr * L.ex, r0 == 0});
        }
        plan.code_off.push_back(off);
        off += pad16(int64_t(w) * d.m);
        plan.blocks.push_back(d);
      }
    }
  }
  plan.item_start.push_back(int32_t(plan.items.size()));
  plan.codes_bytes = off;
}

std::vector<uint8_t> write_header(const Problem& p, int64_t nblocks,
                                  const std::vector<std::vector<uint8_t>>& bits,
                                  const std::vector<StreamHeader::Batch>& batches, uint32_t extra) {
  std::vector<uint8_t> planb;
  for (int v = 0; v < p.nvars; ++v) {
    const std::vector<uint8_t> empty;
    const auto& b = (p.flags & 1) ? bits[v] : empty;
    put<uint32_t>(planb, uint32_t(b.size()));
    std::vector<uint8_t> packed((b.size() + 7) / 8, 0);
    for (size_t i = 0; i < b.size(); ++i)
      if (b[i]) packed[i >> 3] |= uint8_t(1u << (i & 7));
    planb.insert(planb.end(), packed.begin(), packed.end());
  }
  uint32_t hdr = uint32_t(kFixed + 8 * p.nvars + planb.size() + 24 * batches.size());
  std::vector<uint8_t> out;
  out.reserve(hdr);
  out.insert(out.end(), {'D', 'L', 'S', '1'});
  put<uint32_t>(out, kVersion);
  put<uint32_t>(out, hdr);
  put<uint32_t>(out, (p.flags & 1) | ((p.flags & DLS_L2) ? 2u : 0u) | ((p.flags & DLS_GLOBAL) ? 4u : 0u));
  put<int32_t>(out, p.ndim());
  put<int32_t>(out, p.nvars);
  put<int32_t>(out, p.dtype);
  put<int32_t>(out, p.r_max);
  put<int64_t>(out, p.nx);
  put<int64_t>(out, p.ny);
  put<int64_t>(out, p.nz);
  put<int64_t>(out, p.nt);
  put<int32_t>(out, p.px);
  put<int32_t>(out, p.py);
  put<int32_t>(out, p.pz);
  put<int32_t>(out, p.pmin);
  put<int32_t>(out, p.window);
  put<int32_t>(out, kBatchBlocks);
  put<uint64_t>(out, uint64_t(nblocks));
  put<uint32_t>(out, uint32_t(batches.size()));
  put<uint32_t>(out, extra);
  for (int v = 0; v < p.nvars; ++v) put<double>(out, p.eps[v]);
  out.insert(out.end(), planb.begin(), planb.end());
  for (const auto& b : batches) {
    put<uint64_t>(out, b.off);
    put<uint64_t>(out, b.csize);
    put<uint64_t>(out, b.usize);
  }
  return out;
}

std::string parse_header(const uint8_t* buf, size_t n, StreamHeader& h) {
  if (buf == nullptr || n < kFixed) return "stream shorter than the fixed header";
  if (std::memcmp(buf, "DLS1", 4) != 0) return "bad magic";
  if (get<uint32_t>(buf + 4) != kVersion) return "unsupported version";
  uint32_t hdr = get<uint32_t>(buf + 8);
  uint32_t flags = get<uint32_t>(buf + 12);
  Problem& p = h.prob;
  int ndim = get<int32_t>(buf + 16);
  p.nvars = get<int32_t>(buf + 20);
  p.dtype = get<int32_t>(buf + 24);
  p.r_max = get<int32_t>(buf + 28);
  p.nx = get<int64_t>(buf + 32);
  p.ny = get<int64_t>(buf + 40);
  p.nz = get<int64_t>(buf + 48);
  p.nt = get<int64_t>(buf + 56);
  p.px = get<int32_t>(buf + 64);
  p.py = get<int32_t>(buf + 68);
  p.pz = get<int32_t>(buf + 72);
  p.pmin = get<int32_t>(buf + 76);
  p.window = get<int32_t>(buf + 80);
  int bb = get<int32_t>(buf + 84);
  h.nblocks = int64_t(get<uint64_t>(buf + 88));
  uint32_t nbatches = get<uint32_t>(buf + 96);
  p.flags = (flags & 1) | ((flags & 2) ? uint32_t(DLS_L2) : 0u) | ((flags & 4) ? uint32_t(DLS_GLOBAL) : 0u);
  h.extra = get<uint32_t>(buf + 100);
  if (flags & ~7u) return "unknown stream flags";
  p.precision = 0;
  if (hdr > n || hdr < kFixed) return "bad header length";
  if (p.nvars < 1 || p.nvars > 65536 || (p.dtype != 0 && p.dtype != 1) || bb != kBatchBlocks)
    return "bad header fields";
  if (p.nx < 1 || p.ny < 1 || p.nz < 1 || p.nt < 1 || p.window < 1 || p.window > 32 ||
      p.px < 1 || p.px > 32 || p.py < 1 || p.py > 32 || p.pz < 1 || p.pz > 32 ||
      p.r_max < 1 || p.r_max > 32 || ndim != p.ndim())
    return "bad sizes";
  if ((p.flags & 1) && (!is_pow2(p.px) || !is_pow2(p.pmin) || p.pmin > p.px))
    return "bad adaptive sizes";
  if (p.nx > (int64_t(1) << 31) || p.ny > (int64_t(1) << 31) || p.nz > (int64_t(1) << 31) ||
      p.nt > (int64_t(1) << 31))
    return "bad sizes";
  // the value count, without overflow: at most 2^50
  {
    const double vals = double(p.nvars) * double(p.nt) * double(p.nz) * double(p.ny) * double(p.nx);
    if (!(vals <= double(int64_t(1) << 50))) return "grid too large";
  }
  if (h.nblocks < 1 || h.nblocks > p.values()) return "bad block count";
  size_t pos = kFixed;
  if (pos + 8 * size_t(p.nvars) > hdr) return "truncated bounds";
  p.eps.resize(p.nvars);
  for (int v = 0; v < p.nvars; ++v) {
    p.eps[v] = get<double>(buf + pos);
    pos += 8;
    if (!(p.eps[v] > 0.0) || !(p.eps[v] < 1e300)) return "bad bound";
  }
  h.bits.assign(p.nvars, {});
  for (int v = 0; v < p.nvars; ++v) {
    if (pos + 4 > hdr) return "truncated plan";
    uint32_t nb = get<uint32_t>(buf + pos);
    pos += 4;
    size_t nbyte = (size_t(nb) + 7) / 8;
    if (pos + nbyte > hdr) return "truncated plan bits";
    h.bits[v].resize(nb);
    for (uint32_t i = 0; i < nb; ++i) h.bits[v][i] = (buf[pos + (i >> 3)] >> (i & 7)) & 1;
    pos += nbyte;
  }
  if (pos + 24 * size_t(nbatches) != hdr) return "header length mismatch";
  // the global-basis mode appends one basis batch per variable
  const int64_t want = (h.nblocks + kBatchBlocks - 1) / kBatchBlocks + ((p.flags & DLS_GLOBAL) ? p.nvars : 0);
  if (int64_t(nbatches) != want) return "batch count mismatch";
  if (p.flags & DLS_GLOBAL) {
    if ((p.flags & (DLS_L2 | 1u)) || p.window != 1 || int64_t(p.px) * p.py * p.pz > 1024 || p.px > p.nx ||
        p.py > p.ny || p.pz > p.nz || h.extra > 2)
      return "bad global-basis header";
  }
  h.batches.resize(nbatches);
  for (uint32_t i = 0; i < nbatches; ++i) {
    h.batches[i].off = get<uint64_t>(buf + pos);
    h.batches[i].csize = get<uint64_t>(buf + pos + 8);
    h.batches[i].usize = get<uint64_t>(buf + pos + 16);
    pos += 24;
    if (h.batches[i].off > n || h.batches[i].csize > n - hdr ||
        h.batches[i].off > n - hdr - h.batches[i].csize)
      return "batch beyond end of stream";
  }
  h.header_bytes = hdr;
  return "";
}

std::string plan_from_header(const StreamHeader& h, Plan& pl, int slice) {
  const Problem& p = h.prob;
  // the block count of a uniform plan (for an adaptive plan: its roots, a
  // lower bound), from the sizes alone, before any leaf is built: a corrupt
  // header must not make the parser allocate its grid
  {
    const double per = double((p.nx + p.px - 1) / p.px) * double((p.ny + p.py - 1) / p.py) *
                       double((p.nz + p.pz - 1) / p.pz);
    const double nb = double(p.nvars) * double((p.nt + p.window - 1) / p.window) * per;
    if ((p.flags & DLS_ADAPTIVE) ? nb > double(h.nblocks) : nb != double(h.nblocks)) return "block count mismatch";
  }
  if (h.nblocks > (int64_t(1) << 31)) return "too many blocks";
  pl.leaves.assign(p.nvars, {});
  pl.bits = h.bits;
  for (int v = 0; v < p.nvars; ++v) {
    if (p.flags & DLS_ADAPTIVE) {
      bool ok = true;
      pl.leaves[v] = leaves_from_bits(p, h.bits[v], &ok);
      if (!ok) return "split bits inconsistent with the grid";
    } else {
      if (!h.bits[v].empty()) return "split bits in a uniform stream";
      pl.leaves[v] = uniform_leaves(p);
    }
  }
  int64_t nb = 0;
  for (int v = 0; v < p.nvars; ++v) nb += int64_t(pl.leaves[v].size()) * ((p.nt + p.window - 1) / p.window);
  if (nb != h.nblocks) return "block count mismatch";
  build_blocks(p, pl, slice);
  return "";
}

}  // namespace dls
