// Internal declarations shared by the libdls host code and kernels.
//
// Device layout (all buffers owned by a dls_ctx):
//   desc[b]        BlockDesc, blocks ordered variable, window, patch (z, y, x)
//   items[i]       a slice of one block's points, the unit of work of the
//                  Gram and encode kernels; a block's items are contiguous
//   codes          per block: one byte per value, the zigzag int8 residual
//                  codes (0xFF = escape), [t][p] order, padded to 16 bytes;
//                  block regions start 16-byte aligned
//   qv / qa        per block: 4 byte planes of zigzag int32 codes of the
//                  quantized basis qV[k][t] / coefficients qA[k][p], each
//                  plane padded to 16 bytes
//   escapes        (key, value bits) pairs appended by the encode kernel:
//                  key = block << 32 | (t * M_b + p)
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#if defined(__HIPCC__)
#define DLS_HD __host__ __device__
#else
#define DLS_HD
#endif

namespace dls {

constexpr int kBasisBits = 16;       // qV = rint(V * 2^16)
constexpr int kResShift = 17;        // 2 eps = 2^17 * (eps * 2^-16)
constexpr uint8_t kEscCode = 0xFF;  // residual code of an escaped point
constexpr int kQLimit = 127;         // |q| above this is an escape
constexpr int kBatchBlocks = 1000;   // Sec. 2.7.2: batches of 1000 patches
constexpr double kKappa = 1.0;       // tau = kappa eps^2 M_b W_b
constexpr int kZlibLevel = 6;

DLS_HD inline int64_t pad16(int64_t n) { return (n + 15) & ~int64_t(15); }

// 32 bytes; mirrored by dls_encode_info.d_desc
struct BlockDesc {
  int32_t x0, y0, z0, t0;
  int32_t ext;    // px | py << 8 | pz << 16 | w << 24
  int32_t var;
  int32_t m;      // px * py * pz
  int32_t vec;    // 1 if rows are 16-byte aligned runs of 4k elements
  DLS_HD int px() const { return ext & 0xFF; }
  DLS_HD int py() const { return (ext >> 8) & 0xFF; }
  DLS_HD int pz() const { return (ext >> 16) & 0xFF; }
  DLS_HD int w() const { return (ext >> 24) & 0xFF; }
};
static_assert(sizeof(BlockDesc) == 32, "BlockDesc layout");

struct Item {
  int32_t block;
  int32_t p0;     // first point (multiple of px)
  int32_t np;     // number of points
  int32_t first;  // 1 for the block's first item
};

struct Dims {
  int64_t nx, ny, nz, nt;
};

struct Problem {               // validated copy of dls_params
  int nvars;
  int64_t nx, ny, nz, nt;
  int dtype;                   // 0 f32, 1 f64
  int px, py, pz, pmin, window, r_max;
  int precision;
  uint32_t flags;
  int basis = 0;               // global-basis mode: dls_basis_kind
  uint64_t seed = 0;           // global-basis mode: learning-patch draws
  std::vector<double> eps;
  int ndim() const { return nz > 1 ? 3 : 2; }
  int esize() const { return dtype == 0 ? 4 : 8; }
  int wpad() const { return window <= 16 ? 16 : 32; }
  int64_t values() const { return int64_t(nvars) * nt * nz * ny * nx; }
};

struct Leaf {
  int32_t x0, y0, z0, ex, ey, ez;
};

// Plan: leaves per variable, block list, items and static code offsets.
struct Plan {
  std::vector<std::vector<Leaf>> leaves;   // per variable
  std::vector<std::vector<uint8_t>> bits;  // per variable split bits (adaptive)
  std::vector<BlockDesc> blocks;
  std::vector<Item> items;
  std::vector<int32_t> item_start;         // [nblocks + 1]
  std::vector<int64_t> code_off;           // [nblocks]
  int64_t codes_bytes = 0;
};

std::vector<Leaf> uniform_leaves(const Problem& p);
std::vector<Leaf> leaves_from_bits(const Problem& p, const std::vector<uint8_t>& bits, bool* ok);
void build_blocks(const Problem& p, Plan& plan, int slice_points);

// ---- stream format (header + batch table + zlib streams) ----
struct StreamHeader {
  Problem prob;
  int64_t nblocks = 0;
  std::vector<std::vector<uint8_t>> bits;
  struct Batch { uint64_t off, csize, usize; };
  std::vector<Batch> batches;
  size_t header_bytes = 0;
  uint32_t extra = 0;   // global-basis mode: the basis kind
};

// Returns "" on success, else a message (stream is corrupt).
std::string parse_header(const uint8_t* buf, size_t n, StreamHeader& h);
// Rebuild the plan of a parsed header (leaves, blocks, items); "" on success.
std::string plan_from_header(const StreamHeader& h, Plan& pl, int slice);
std::vector<uint8_t> write_header(const Problem& p, int64_t nblocks,
                                  const std::vector<std::vector<uint8_t>>& bits,
                                  const std::vector<StreamHeader::Batch>& batches, uint32_t extra = 0);

}  // namespace dls
