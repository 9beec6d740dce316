// Shared pieces of the Ozaki-split products (DD: ozaki.hip, QD:
// ozaki_qd.hip): the workspace layout of the INT8 slice stacks and the two
// preparation launches (exponents, slicing) in ozaki_split.hip.
#pragma once
#include "common.hpp"

namespace ddqd {

constexpr int kOzFrag = 1024;  // bytes of one 32x32 INT8 fragment block

// Slice stacks of one batch entry: for every 32-line block (rows of A,
// columns of B) and 32-k block, S fragments of 1 KB in the order of the
// 32x32x32 MFMA (lane l: line l % 32, k = 16 (l / 32) + 0..15).
struct OzLayout {
  int64_t m, n, l;
  int64_t rb, cb, kb;  // 32-blocks: rows of A, columns of B, K
  int S;
  int64_t a_bytes, b_bytes;  // per batch entry
};

// DD products use 64x64 tiles (rb, cb even), QD products 32x32 blocks.
inline OzLayout oz_layout(int P, int64_t m, int64_t n, int64_t l, int S) {
  OzLayout o;
  o.m = m;
  o.n = n;
  o.l = l;
  o.S = S;
  o.rb = P == 2 ? ((m + 63) / 64) * 2 : (m + 31) / 32;
  o.cb = P == 2 ? ((n + 63) / 64) * 2 : (n + 31) / 32;
  o.kb = (l + 31) / 32;
  o.a_bytes = o.rb * o.kb * S * (int64_t)kOzFrag;
  o.b_bytes = o.cb * o.kb * S * (int64_t)kOzFrag;
  return o;
}

inline size_t oz_align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of one Ozaki product (batch entries): the slice stacks of A and
// B, the row exponents of A (rb * 32 ints per entry), the column exponents of
// B (cb * 32) and the column maxima's exponents per 32-row slab of B
// (kb * cb * 32).
struct OzWs {
  signed char *Asl, *Bsl;
  int *ea, *fb, *part;
};
inline size_t oz_workspace_bytes(const OzLayout& o, int64_t batch) {
  return oz_align256(o.a_bytes * batch) + oz_align256(o.b_bytes * batch) +
         oz_align256(sizeof(int) * (size_t)(batch * (o.rb + o.cb) * 32)) +
         oz_align256(sizeof(int) * (size_t)(batch * o.kb * o.cb * 32));
}
inline OzWs oz_ws(char* ws, const OzLayout& o, int64_t batch) {
  OzWs w;
  w.Asl = (signed char*)ws;
  ws += oz_align256(o.a_bytes * batch);
  w.Bsl = (signed char*)ws;
  ws += oz_align256(o.b_bytes * batch);
  w.ea = (int*)ws;
  w.fb = w.ea + batch * o.rb * 32;
  ws += oz_align256(sizeof(int) * (size_t)(batch * (o.rb + o.cb) * 32));
  w.part = (int*)ws;
  return w;
}

// Unrelated DD Ozaki products of one grouped launch (kernel argument, under
// the 4 KB limit): each problem with its own layout and workspace; the
// prefix sums give problem p the exponent workgroups [wg[p], wg[p+1]), the
// slicing chunks [chunk[p], chunk[p+1]) and the product tiles
// [tile[p], tile[p+1]) of the concatenated lists.
constexpr int kOzGroup = 12;
struct OzProb {
  GemmBatch g;  // batch = 1
  OzLayout o;
  OzWs w;
};
struct OzGroupArgs {
  int count;
  OzProb p[kOzGroup];
  int64_t wg[kOzGroup + 1], chunk[kOzGroup + 1], tile[kOzGroup + 1];
};
static_assert(sizeof(OzGroupArgs) <= 4096, "kernel argument limit");

// Problem q of a grouped launch owning item x of the prefix sums `start`.
__device__ __forceinline__ int oz_group_find(const int64_t* start, int count, int64_t x) {
  int q = 0;
  while (q + 1 < count && x >= start[q + 1]) q++;
  return q;
}

// Exponent workgroups and slicing chunks of one product (grouped launches).
inline int64_t oz_exp_wgs(const OzLayout& o) {
  return (o.rb * 32 + 3) / 4 + ((o.cb * 32 + 63) / 64) * o.kb;
}
// 32-k blocks per slicing chunk (DD: four, QD: two) and chunks per product.
constexpr int oz_slice_kb(int P) { return P == 2 ? 4 : 2; }
inline int64_t oz_slice_chunks(const OzLayout& o, int P) {
  const int kb = oz_slice_kb(P);
  return (o.rb + o.cb) * ((o.kb + kb - 1) / kb);
}

// The three launches of a group (exponents, slicing, products), P = 2.
int launch_oz_exponents_grouped(const OzGroupArgs& ga, hipStream_t s);
int launch_oz_slice_grouped(const OzGroupArgs& ga, int S, hipStream_t s);

// Exponents e with max |leading component| < 2^(e - 1): of A's rows into
// w.ea (an all-zero row, and every padded row, gets 1: its digits are all
// zero, so any exponent gives the same result), and of B's columns per 32-row
// slab into w.part (an all-zero slab gets a sentinel far below any exponent,
// so the column's maximum over slabs ignores it).  One launch.
int launch_oz_exponents(const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s);

// The S digits of every scaled entry of A and B (P = 2 DD, 4 QD); also
// reduces the slab exponents of B into w.fb, which the product reads.
int launch_oz_slice(int P, const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s);

}  // namespace ddqd
