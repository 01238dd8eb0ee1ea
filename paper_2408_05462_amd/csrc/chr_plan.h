// chr_plan.h -- launch plans of the compress / reconstruct / extract paths.
#pragma once

#include "chr_device.h"
#include "scan.h"

namespace chr {

constexpr int kMaxLevels = 16;
constexpr int kSumSegs = 8;      // workgroups that checksum one block's stream bytes

// Statistics of the points one workgroup encoded (ordered images of
// binary32 values; counts cover the points the block owns).
struct Part {
  uint32_t rmin, rmax;   // reconstructed values (block index)
  uint32_t xmin, xmax;   // input values (header range)
  uint32_t nonfinite, nO, nC, pad;
};

// Compression: per-level chunk slots hold one 64-point chunk each before the
// stream is assembled (width/exact counts, packed codes, exact mask, exact
// values); slots of level l for block b start at slot_base[l] + b*maxch[l],
// or, for merged units (their sizes differ), at ubase[b*nL + nL-1-l].
// Workgroups per block of the block-activity pass (differentiated error
// control); the workspace holds 2 partial keys per block and workgroup.
constexpr int kActSplit = 16;

struct EncPlan {
  Geo g;
  L0Geo l0;
  int cpw0;                      // level-0 chunks per wave (tile shape; results do not depend on it)
  int tile0;                     // level 0 by plane pairs (64-cell blocks; results do not depend on it)
  int tile1;                     // level 1 likewise
  int top;                       // levels L .. 2 of a 64-cell block in one workgroup, in LDS
  int64_t slot_base[kMaxLevels];
  uint32_t maxch[kMaxLevels];
  int64_t nslots;
  int64_t gd[kMaxLevels][3];     // compact grid dims of level l
  int64_t g_off[kMaxLevels];     // offset (floats) of compact grid l >= 1 in G
  uint64_t payload_off;          // bytes before the first section
  uint64_t cap;
  const float *x;
  float *G;
  U4 *cnt, *P;                   // per-slot {w, has exact, #exact, 0} and exclusive prefix
  uint32_t *pay;                 // nslots * 32 words
  unsigned long long *emask;     // nslots
  float *exv;                    // nslots * 64
  Part *part;                    // per block: part_per_block workgroup records
  int64_t part_per_block;        // records per block: level-0, level-1 and level-2 workgroups, coarse levels
  int64_t part_l1;               // first level-1 record of a block
  int64_t part_l2;               // first level-2 record of a block
  int l2fast;                    // level 2 runs in its own wide kernel (else with the coarse levels)
  Part *bst;                     // per block reduction of its records
  uint32_t *csum;                // per block, kSumSegs partial checksums of its byte range
  int64_t pack_base[kMaxLevels]; // first packing workgroup of each level
  int64_t pack_gpb[kMaxLevels];  // packing workgroups per block and level
  uint64_t *secsz, *secoff;      // nblocks*nL (+1)
  uint8_t *out;
  void *result;                  // chr_result*
  int32_t *codes;
  uint8_t *flags;
  uint32_t *act;                 // per block: 1 = active (differentiated error control only)
  const int64_t *ubase;          // merged units: first slot of every (unit, level), levels from the coarsest
};

// First chunk slot of level l of storage unit b.
__device__ inline int64_t slot_of(const EncPlan &P, int l, int64_t b) {
  if (P.ubase) return P.ubase[b * P.g.nL + (P.g.nL - 1 - l)];
  return P.slot_base[l] + b * (int64_t)P.maxch[l];
}

// Reconstruction of levels L..lo.
struct DecPlan {
  Geo g;
  L0Geo l0;
  int cpw0;                      // level-0 chunks per wave: 8, 16, 32 or 64
  int tile0;                     // level 0 of 64-cell blocks by plane pairs (results do not depend on it)
  int lo;
  int64_t gd[kMaxLevels][3];
  float *gp[kMaxLevels];         // compact grid of level l (gp[lo] = output when lo >= 1)
  const uint8_t *s;
  uint64_t sbytes;
  uint64_t payload_off;
  float *out;                    // full-resolution output when lo == 0
  int32_t *status;
  int prune;                     // reconstruct only blocks that can hold an isosurface for k in [kmin, kmax]
  float kmin, kmax;
  // below-isovalue bits of the level-0 output (marching cubes' words: 64
  // points along x per u64, rows (z, y)), one plane of bplane words per
  // isovalue kb[0..nk) (bits == nullptr: none)
  unsigned long long *bits;
  int64_t bplane, bnw;
  int nk;
  float kb[kMaxIso];
};

struct McPlan {
  int64_t n[3];
  int64_t nrows, nw;             // point rows (nz*ny) and 64-bit words per row
  float k, spacing;
  const float *f;
  unsigned long long *bits;      // nrows * nw below-isovalue bits
  uint32_t *cnt;                 // per word {vertices, triangles, crossing points, active cells}, packed (scan.h)
  U4 *P;                         // their exclusive prefix
  uint32_t *vlist;               // crossing points (word*64 + bit), cap_pv entries
  uint32_t *clist;               // active cells (word*64 + bit), cap_ac entries
  uint32_t *tb;                  // first triangle id of every 256th active cell, cap_ac / 256 + 1 entries
  int64_t cap_pv, cap_ac;
  float *verts;
  int32_t *tris;
  int64_t cap_v, cap_t;
  int64_t *counts;
  uint8_t *cases;
  FastDiv d_nw, d_n1;            // word -> (row, word in row), row -> (z, y); set by the launchers
  uint32_t org[3];               // grid coordinates (z, y, x) of point 0 in a larger field (0: the field itself)
  int64_t py, pz;                // elements between rows and between planes of f (n[2] and n[1]*n[2] for a whole field)
};

// Measurement hook: records a HIP event around launches of the kernel
// selected with chr_prof_enable (no-op otherwise).
void prof_mark(const char *kernel, hipStream_t s, int end);

// launchers (encode.hip, decode.hip, mc.hip)
// Index signature of every block into p.act[0 .. nblocks) (block merging).
void launch_block_signatures(const EncPlan &p, hipStream_t s);
void launch_encode(const EncPlan &p, int64_t scan_tmp_elems_u4, U4 *scan_tmp, uint64_t *scan_tmp64,
                   hipStream_t s);
int64_t encode_fine_groups(const EncPlan &p);   // level-0 workgroups per block
bool encode_tile0_ok(const EncPlan &p);         // level 0 can run by plane pairs
bool encode_tile1_ok(const EncPlan &p);         // level 1 can run by plane pairs
bool encode_top_ok(const EncPlan &p);           // levels L .. 2 can run in one workgroup per block
int64_t encode_tile0_groups(const EncPlan &p);  // plane pairs per block
int64_t encode_l1_groups(const EncPlan &p);     // level-1 workgroups per block
int64_t encode_l2_groups(const EncPlan &p);     // level-2 workgroups per block (records reserved)
bool encode_l2_fast(const EncPlan &p);          // whether level 2 runs in its own wide kernel
void encode_pack_layout(EncPlan &p);            // fills pack_base / pack_gpb
void launch_decode(const DecPlan &p, hipStream_t s);
bool decode_tile0_used(const DecPlan &p);      // level 0 by plane pairs (writes p.bits when set)
void launch_status_reset(int32_t *status, hipStream_t s);  // *status = 0 by a kernel (capturable)
void launch_mc(const McPlan &p, U4 *scan_tmp, hipStream_t s);        // count + emit
void launch_mc_count(const McPlan &p, U4 *scan_tmp, hipStream_t s);  // bits, counts, scan; totals to counts[0..3]
void launch_mc_emit(const McPlan &p, hipStream_t s);                 // lists, vertices, triangles, counts[0..1]
void launch_mc_cases(const McPlan &p, hipStream_t s);
void launch_mc_bits(const McPlan &p, hipStream_t s);                 // the bits of isovalue p.k into p.bits
void launch_mc_from_bits(const McPlan &p, U4 *scan_tmp, hipStream_t s); // count + emit from p.bits
void launch_range(const float *f, int64_t n, float *out, hipStream_t s);
size_t topo_workspace_bytes();
int launch_topology(const float *f, const int64_t dims[3], const float *iso, int K, int64_t nth, double *out,
                    void *ws, hipStream_t s);
void mc_table_host(uint8_t *ntri, int8_t *tri);

// plans travel as kernel arguments (at most 4 KiB)
static_assert(sizeof(EncPlan) <= 4096 && sizeof(DecPlan) <= 4096 && sizeof(McPlan) <= 4096,
              "a plan must fit the kernel argument space");

}  // namespace chr
