// ccwsim_common.h -- helpers shared by the CCWSIM HIP kernels and their host
// launchers: the counter-based random numbers, the keyed tie-break
// bijection (and its inverse), candidate keys and the problem geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CCW_HD __host__ __device__ __forceinline__

namespace ccw {

// ---------------------------------------------------------------------------
// Random numbers.  Every draw of the method (path corner, tie-break key, the
// uniform pick among the K best) is a pure function of (seed, stream, a, b),
// so results do not depend on the order in which patches run.  The mixer is
// SplitMix64 (Steele, Lea, Flood 2014): golden-ratio increment followed by
// its 64-bit finaliser; further words are folded in with one more round.
// ---------------------------------------------------------------------------
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;
constexpr uint64_t kStreamPath = 1, kStreamTiebreak = 2, kStreamDraw = 3;

CCW_HD uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

CCW_HD uint64_t draw64(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  uint64_t h = mix64(seed + kGolden);
  h = mix64((h ^ stream) + kGolden);
  h = mix64((h ^ a) + kGolden);
  h = mix64((h ^ b) + kGolden);
  return h;
}

// ---------------------------------------------------------------------------
// Keyed bijection on [0, 2^20) ordering equal scores.  Rounds: xor a key
// word, multiply by an odd constant mod 2^20, xor-shift right.  The inverse
// undoes each round in reverse order.
// ---------------------------------------------------------------------------
constexpr uint32_t kMask20 = 0xFFFFFu;
constexpr uint32_t kMulA = 0x6B5A5u, kMulB = 0x3A8F3u;

constexpr uint32_t inv_odd20(uint32_t a) {
  // Newton iteration for the inverse of an odd number mod 2^20
  uint32_t x = a;
  for (int i = 0; i < 5; ++i) x = (x * (2u - a * x)) & kMask20;
  return x;
}
constexpr uint32_t kInvA = inv_odd20(kMulA), kInvB = inv_odd20(kMulB);
static_assert(((kMulA * kInvA) & kMask20) == 1u, "inverse of A");
static_assert(((kMulB * kInvB) & kMask20) == 1u, "inverse of B");

// Low 32 bits of a product of two values below 2^24 (both operands here
// are below 2^20, so the low 20 bits are those of the full product); on the
// GPU this is the full-rate 24-bit multiply.
CCW_HD uint32_t mul_lo24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul24(a, b);
#else
  return a * b;
#endif
}

CCW_HD uint32_t tie_perm(uint32_t x, uint64_t key) {
  const uint32_t k1 = (uint32_t)(key & kMask20);
  const uint32_t k2 = (uint32_t)((key >> 20) & kMask20);
  const uint32_t k3 = (uint32_t)((key >> 40) & kMask20);
  x = (x & kMask20) ^ k1;
  x = mul_lo24(x, kMulA) & kMask20;
  x ^= x >> 10;
  x ^= k2;
  x = mul_lo24(x, kMulB) & kMask20;
  x ^= x >> 9;
  return (x ^ k3) & kMask20;
}

CCW_HD uint32_t tie_perm_inv(uint32_t y, uint64_t key) {
  const uint32_t k1 = (uint32_t)(key & kMask20);
  const uint32_t k2 = (uint32_t)((key >> 20) & kMask20);
  const uint32_t k3 = (uint32_t)((key >> 40) & kMask20);
  uint32_t x = (y & kMask20) ^ k3;
  x = x ^ (x >> 9) ^ (x >> 18);  // undo x ^= x >> 9 on 20 bits
  x = mul_lo24(x, kInvB) & kMask20;
  x ^= k2;
  x = x ^ (x >> 10);             // undo x ^= x >> 10 on 20 bits
  x = mul_lo24(x, kInvA) & kMask20;
  return (x ^ k1) & kMask20;
}

// Candidate key: hard-data mismatch first, then the score, then the tie-break.
CCW_HD uint64_t make_key(uint32_t mismatch, int32_t score, uint32_t tie) {
  const uint64_t m = mismatch > 4095u ? 4095u : mismatch;
  const uint64_t s = (uint64_t)((uint32_t)score ^ 0x80000000u);  // score + 2^31
  return (m << 52) | (s << 20) | (uint64_t)(tie & kMask20);
}

// ---------------------------------------------------------------------------
// Geometry of one problem, passed by value to kernels.
// ---------------------------------------------------------------------------
constexpr int kMaxLevel = 6;

struct Geom {
  int ndim;
  int level;
  int ti[3];       // TI extent
  int np[3];       // TI extent after edge replication to a multiple of b
  int G[3];        // level-J grid (approximation extent)
  int b[3];        // block factor per axis (2^J on used axes, else 1)
  int beta;        // cells per level-J block
  int log2beta;
  int shift;       // S = E - (C << shift): log2beta + 1 for Haar block sums, 1 for 5/3 coefficients
  int wavelet;     // 0 Haar, 1 LeGall 5/3
  int T[3], OV[3], tc[3];       // template, overlap, template in blocks
  int cand[3];     // candidates per axis
  int ncand;
  int sg[3];       // grid extent
  int stride[3], lat[3], pad[3];
  int margin[3];   // virtual-template margin
  int Gj[kMaxLevel + 1][3];     // extent of level j (j = 0 is np)
  long long det_off[kMaxLevel + 2];  // details offset of level j (1-based)
  long long det_total;
  long long tcells, wcells, pcells;
};

// Split a linear index of an e0 x e1 x (..) box into (x, y, z) with 32-bit
// divisions only.
CCW_HD void split3(int i, int e0, int e1, int& x, int& y, int& z) {
  const int e01 = e0 * e1;
  z = i / e01;
  const int r = i - z * e01;
  y = r / e0;
  x = r - y * e0;
}

CCW_HD long long idx3(int x, int y, int z, const int d[3]) {
  return (long long)x + (long long)d[0] * ((long long)y + (long long)d[1] * z);
}

// The same for boxes of fewer than 2^31 cells.
CCW_HD int idx3i(int x, int y, int z, const int d[3]) { return x + d[0] * (y + d[1] * z); }

}  // namespace ccw
