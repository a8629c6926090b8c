// MI355X (gfx950) hot path of the site-based suspension lattice Boltzmann
// method of dos Santos & Philippi, behind the C ABI of include/lbm.h.
//
// One time step is four launches on the caller's stream (five with the
// near-contact closure):
//   sweep      one streaming pass over every site, A -> B (HBM bound; SoA,
//              x fastest, coalesced): pull-propagation of the previous step
//              (whose IS substep is already in A), BGK collision with body
//              force, and the BS substep at owned BS sites (the site's
//              post-collision moments go to the owner entry's slot).
//                                                          eq. 1-5, 12, 3 (left)
//   reduce     one workgroup per particle: momentum dp and angular momentum dl
//              of every owned BS site from its slot (no owner-map lookup:
//              unowned slots carry a mark), deterministic wave-shuffle + LDS
//              sums, the list of particles close enough to collide, and the
//              list of particles whose sites may coincide with this one's
//              after the translation.                                eq. 6-9
//   particles  one workgroup per box: Newton-Euler update with buoyancy-
//              corrected weight, hard-core collisions in lexicographic pair
//              order, translation and integer shift.        eq. 10-11, 13, 16-19
//   prepare    one to eight workgroups per particle: site ownership at the new
//              shifts (lowest particle id among the BS/IS entries on a site,
//              read from the kind grids of the particles that may share it),
//              the IS substep at the new positions (eq. 12) written in place
//              into the post-collision state -- f^eq_i(rho_I, u_p' + omega_p'
//              x r) at every owned IS site -- the flags of the ball sites of a
//              particle whose shift changed (and of the sites it left), and,
//              by the owning entry, the record of every owned BS site: the
//              rigid-body velocity u_p + omega x r of its next BS substep
//              (eq. 5) and the owner entry; a BS entry whose site is held by
//              another particle or a wall marks its slot unowned instead.
// Balls too large for kind grids keep an owner map instead: reduce releases
// it, a stamp launch rebuilds it at the new shifts (eq. 14-15) and prepare
// reads it, one thread per entry.
// The IS substep of step t acts on the post-collision populations of IS sites
// just before they propagate; written into the state, it is what the sweep of
// step t+1 pulls.  Outside every ball the sweep reads one flag byte and
// nothing more.
// The populations are stored as deviations g_i = f_i - w_i rho0 so that the
// momentum differences behind the particle forces survive FP32 storage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "lattice.h"
#include "lbm.h"
#include "mlp_core.h"

namespace {

constexpr int kEmpty = 0x7fffffff;  // map value of a site no entry claims
// drho of the slot of a BS entry that does not own its site (another particle
// or a wall holds it): the entry adds nothing to its particle's sums
constexpr double kSlotUnowned = -0x1p1000;
constexpr int64_t kMaxEntries = (int64_t)1 << 29;  // owner map stores 2e + 1 < kEmpty
constexpr uint8_t kSiteBall = 1;  // site flag: some ball covers the site
constexpr uint8_t kSiteBS = 2;    // site flag: an owned BS site (its record is valid)
constexpr int kCandMax = 64;        // close neighbours listed per particle
constexpr double kMargin = 1.0;     // candidate search margin (lattice units)
// Particles whose site sets could share a site at the new shifts of a step:
// centres within r_i + r_j + kShareMargin at the start of the step.  Each
// centre moves by less than 1/2 in a step (the collision bound) and the
// translated template's centre x0 + k lies within sqrt(3)/2 of the true one,
// so two balls that share a site after the step started closer than
// r_i + r_j + 2 (1/2 + sqrt(3)/2) = r_i + r_j + 2.74.
constexpr double kShareMargin = 3.0;
constexpr int kNbrMax = 128;        // such neighbours listed per particle
constexpr int kSweepBlock = 256;
constexpr int kTileMax = 512;        // widest tile of the ensemble sweep
constexpr int kXcdRun = 4;           // adjacent ensemble tiles per XCD (k_sweep_tiles)
constexpr int kBoundaryBlock = 256;  // reduce workgroup (128 for balls of at most kSmallBall entries)
constexpr int kSmallBall = 512;
constexpr int kPrepareBlock = 256;   // workgroup of the per-particle prepare
constexpr size_t kCacheResidentBytes = (size_t)128 << 20;  // half the 256 MB last-level cache
constexpr int kPrepareLocalMax = 8192;  // bound on one ball's entries for the per-particle prepare
constexpr int kParticleBlock = 1024;   // particle update of a one-box context
constexpr int kBoxParticleBlock = 256; // particle update, per box of an ensemble
constexpr int kStatusCollision = 1;
constexpr int kStatusClosure = 2;     // more close pairs than kClosurePairs
constexpr int kStatusRecord = 4;      // an owned-BS record named no entry of the table
constexpr int kClosurePairs = 1024;   // close pairs one step of the closure handles
constexpr size_t kAlign = 256;

// ---------------------------------------------------------------------------
// Storage traits: compute type and load / streaming store of one population.
// ---------------------------------------------------------------------------
template <typename T>
struct Store;
template <>
struct Store<double> {
  using C = double;
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
  static __device__ __forceinline__ double ldnt(const double* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(double* p, double v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<float> {
  using C = float;
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ float ldnt(const float* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
};
// Half precision: the stored number is g_i / (w_i 2^-10), i.e. the deviation
// normalised by its weight (so that every direction spans the same range of
// O(u) values) and scaled by 2^10 to keep small deviations normal.
template <>
struct Store<_Float16> {
  using C = float;
  static __device__ __forceinline__ float ld(const _Float16* p) { return (float)*p; }
  static __device__ __forceinline__ float ldnt(const _Float16* p) { return (float)__builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(_Float16* p, float v) { __builtin_nontemporal_store((_Float16)v, p); }
};
// bfloat16: the top half of an FP32 number, rounded to nearest even; stores
// g_i / w_i (FP32's exponent range needs no scaling).
struct bf16s {
  uint16_t v;
};
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
// The same rounding on the device, where gfx950 converts in one instruction
// (v_cvt_pk_bf16_f32, round to nearest even); the two agree on every finite
// value.
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__host__ __device__ inline float bf16_bits_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
template <>
struct Store<bf16s> {
  using C = float;
  static __device__ __forceinline__ float ld(const bf16s* p) { return bf16_bits_to_f32(p->v); }
  static __device__ __forceinline__ float ldnt(const bf16s* p) {
    return bf16_bits_to_f32(__builtin_nontemporal_load(&p->v));
  }
  static __device__ __forceinline__ void st(bf16s* p, float v) {
    __builtin_nontemporal_store(bf16_rne(v), (uint16_t*)p);
  }
};

// Multiplier from the stored number to the deviation g_i (1 for FP64/FP32).
template <typename T>
__host__ __device__ constexpr double pop_unit(double w) {
  return std::is_same<T, _Float16>::value ? w * (1.0 / 1024.0) : (std::is_same<T, bf16s>::value ? w : 1.0);
}

// Load / store population i (deviation g_i in the compute type).
template <int Q, typename T>
__device__ __forceinline__ typename Store<T>::C pop_ld(const T* p, int i) {
  using C = typename Store<T>::C;
  return Store<T>::ld(p) * (C)pop_unit<T>(Lattice<Q>::w(i));
}
template <int Q, typename T>
__device__ __forceinline__ void pop_st(T* p, int i, typename Store<T>::C v) {
  using C = typename Store<T>::C;
  Store<T>::st(p, v * (C)(1.0 / pop_unit<T>(Lattice<Q>::w(i))));
}
// The stored number for a plain (not streaming) store: the compute-type value
// the sweep would store (the deviation g_i, or for 16-bit storage g_i /
// (w_i sigma)), rounded to the storage type as Store<T>::st rounds it.
template <typename T>
__device__ __forceinline__ T store_enc(typename Store<T>::C h) {
  if constexpr (std::is_same<T, bf16s>::value)
    return bf16s{bf16_rne(h)};
  else
    return (T)h;
}

// One box of the context: its size, walls, first site in the site arrays
// (boxes of an ensemble are stored one after the other) and one past the id
// of its last particle (the particles of a box have consecutive ids).
struct Geo {
  int nx, ny, nz;
  int64_t N;
  int walls;  // bit a: axis a closed by wall layers 0, 1, n-2, n-1
  int64_t off;
  int p1;
};

struct DevParticles;

// Geometry of every box: the box itself when there is one (kernel argument,
// no load), a device table indexed by the particle's box otherwise.
struct Boxes {
  Geo g0;
  const Geo* tab;
  int nbox;
};

// A site of the wall layers of a closed axis (particles never own these).
__device__ __forceinline__ bool wall_site(const Geo& G, int x, int y, int z) {
  return ((G.walls & 1) && (x < 2 || x >= G.nx - 2)) || ((G.walls & 2) && (y < 2 || y >= G.ny - 2)) ||
         ((G.walls & 4) && (z < 2 || z >= G.nz - 2));
}

struct DevParticles {
  double *x, *x0, *u, *om, *phi, *fext, *dP, *dL, *F, *T;  // [n][3]
  double *m, *I, *rad;                                     // [n]
  int *b0, *k, *org;                                       // [n][3]; org = b0 + k wrapped into the box
  int *ent0, *nbs, *nis, *nin, *cand_n, *jump, *box;       // [n]
  double* fc;                                              // [n][3] closure force of the step
  int *cand;                                               // [n][kCandMax]
  int *pairs;                                              // [n*kCandMax][2]
  // kind grids (per-particle ownership, no owner map in the step):
  int *orgp, *moved;     // [n][3] origin before the last translation; [n] shift changed in it
  int *kg0, *kgR;        // [n] first byte of the particle's kind grid, its half-width R
  int *nbr_n, *nbr;      // [n], [n][kNbrMax]: particles that may share a site with it
  uint8_t* kgrid;        // per particle (2R+1)^d kinds of its template (0 none, 1 BS, 2 IS, 3 interior)
};

__device__ __forceinline__ Geo geo_of(const Boxes& B, const DevParticles& P, int p) {
  return B.nbox == 1 ? B.g0 : B.tab[P.box[p]];
}

struct DevEntries {
  int* off;  // packed int8 offsets x,y,z and kind (1 BS, 2 IS, 3 interior) in the top byte
  int* pid;  // owner particle
};

__host__ __device__ inline int pack_entry(int ox, int oy, int oz, int kind) {
  return (ox & 0xff) | ((oy & 0xff) << 8) | ((oz & 0xff) << 16) | (kind << 24);
}
__device__ __forceinline__ int off_x(int v) { return (int)(int8_t)(v & 0xff); }
__device__ __forceinline__ int off_y(int v) { return (int)(int8_t)((v >> 8) & 0xff); }
__device__ __forceinline__ int off_z(int v) { return (int)(int8_t)((v >> 16) & 0xff); }
__host__ __device__ __forceinline__ int entry_kind(int v) { return (v >> 24) & 0xff; }

__host__ __device__ __forceinline__ int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// v in (-n, 2n) back into [0, n)
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Coordinates of a template offset at the particle's current shift b0 + k
// (offsets are shorter than the box, so one wrap suffices).
__device__ __forceinline__ void entry_xyz(const DevParticles& P, const Geo& G, int p, int pk, int& x, int& y,
                                          int& z) {
  x = wrap1(P.org[3 * p] + off_x(pk), G.nx);
  y = wrap1(P.org[3 * p + 1] + off_y(pk), G.ny);
  z = wrap1(P.org[3 * p + 2] + off_z(pk), G.nz);
}

__device__ __forceinline__ int site_of(const Geo& G, int x, int y, int z) {
  return (int)G.off + x + G.nx * (y + G.ny * z);
}

// ---------------------------------------------------------------------------
// Ball sites.  flag[s] is 0 outside every ball, kSiteBall inside one and
// kSiteBS at an owned BS site; there the site's record vel[4s..4s+2] is the
// rigid-body velocity of its next BS substep and vel[4s+3] the index of the
// owning BS entry, whose slot receives the site's post-collision moments.
// The sweep reads the one-byte flag of every site and the record of BS sites
// only, so it never waits on a map lookup before its own pulls.
// ---------------------------------------------------------------------------
template <typename T>
struct SiteArgs {
  const uint8_t* flag;              // [site]: 0, kSiteBall or kSiteBS
  const typename Store<T>::C* vel;  // [site][4]: record of a kSiteBS site
  double* slot;                     // [entry][4]: post-collision drho, j of an owned BS site
  typename Store<T>::C* drho;       // density deviation of every ball site (this sweep)
  int nent;                         // entries in the table: a record's index must lie below
  int* status;                      // device status word (kStatusRecord)
};

// One site record as a single 16- (FP32) or 32-byte (FP64) load.
__device__ __forceinline__ float4 ld_rec(const float* p) { return *(const float4*)p; }
__device__ __forceinline__ double4 ld_rec(const double* p) { return *(const double4*)p; }

// An entry index carried in a velocity record's fourth slot (bit pattern in
// FP32, exact value in FP64).
template <typename C>
__device__ __forceinline__ C idx_as(int v) {
  if constexpr (std::is_same<C, float>::value)
    return __int_as_float(v);
  else
    return (C)v;
}
template <typename C>
__device__ __forceinline__ int as_idx(C v) {
  if constexpr (std::is_same<C, float>::value)
    return __float_as_int(v);
  else
    return (int)v;
}

// Where the state between two steps keeps population i (eq. 3 splits a step
// into collision and propagation; the state is one of the two halves):
//  kLayAB:       two arrays; the current one holds the post-collision f*_i(x)
//                at [i][x], the sweep pulls f*_i(x - c_i) and writes the other.
//  kLayAAStream: one array (AA pattern) holding the post-propagation f_i(x) at
//                [i][x] (after an odd step, and initially); the sweep reads
//                its own site and writes f*_i(x) to [opp(i)][x].
//  kLayAASwap:   one array holding f*_i(x) at [opp(i)][x] (after an even
//                step); the sweep reads [opp(i)][x - c_i] and writes f*_i(x)
//                to [i][x + c_i], where the next sweep finds it at its own site.
// In both AA halves every thread reads and writes the same q locations.
constexpr int kLayAB = 0, kLayAAStream = 1, kLayAASwap = 2;

// ---------------------------------------------------------------------------
// K1: one pass over every site = propagation of the previous step (pull; the
// previous step's IS substep is already in the state it pulls from), BGK
// collision with body force (eq. 1-3), and the BS substep at owned BS sites
// (eq. 5-7) with the post-collision moments written to the owner's slot.
// ---------------------------------------------------------------------------
template <int Q, typename C>
struct SweepArgs {
  int nx, ny, nz, nxb;
  C omega;   // 1 / tau
  C rho0;
  C fbt[Q];  // 3 w_i c_i . f_b
  int walls;           // bit a: axis a closed by wall layers
  C wu[3][2][3];       // wall velocity [axis][low, high][component]
};

// Velocity of the wall whose layers hold (x, y, z), the lowest closed axis
// deciding at edges; false for a fluid site.  Selects, not indexing, so the
// kernel-argument array stays in scalar registers.
template <int Q, typename C>
__device__ __forceinline__ bool wall_velocity(const SweepArgs<Q, C>& a, int x, int y, int z, int nx, int ny,
                                              int nz, C& vx, C& vy, C& vz) {
  int ax, hi;
  if ((a.walls & 1) && (x < 2 || x >= nx - 2)) {
    ax = 0;
    hi = x >= nx - 2;
  } else if ((a.walls & 2) && (y < 2 || y >= ny - 2)) {
    ax = 1;
    hi = y >= ny - 2;
  } else if ((a.walls & 4) && (z < 2 || z >= nz - 2)) {
    ax = 2;
    hi = z >= nz - 2;
  } else {
    return false;
  }
  vx = ax == 0 ? (hi ? a.wu[0][1][0] : a.wu[0][0][0]) : ax == 1 ? (hi ? a.wu[1][1][0] : a.wu[1][0][0])
                                                               : (hi ? a.wu[2][1][0] : a.wu[2][0][0]);
  vy = ax == 0 ? (hi ? a.wu[0][1][1] : a.wu[0][0][1]) : ax == 1 ? (hi ? a.wu[1][1][1] : a.wu[1][0][1])
                                                               : (hi ? a.wu[2][1][1] : a.wu[2][0][1]);
  vz = ax == 0 ? (hi ? a.wu[0][1][2] : a.wu[0][0][2]) : ax == 1 ? (hi ? a.wu[1][1][2] : a.wu[1][0][2])
                                                               : (hi ? a.wu[2][1][2] : a.wu[2][0][2]);
  return true;
}

// Population layout: blocks of kPopBlock consecutive sites, each block
// holding its q populations one after another: [N / kPopBlock][q][kPopBlock],
// N the sites rounded up to whole blocks.  The q pieces a row of the 256^3
// box writes then lie within one block of 8 rows, and the pieces it pulls
// within the blocks of its own plane and the two next to it, instead of q
// planes apart.  Whole FP32 256^3 step with 500 spheres, by block size:
// planes 0.474 ms, 256 sites 0.472, 1024 0.470, 1536 0.469, 2048 0.456,
// 3072 0.464, 4096 and 8192 0.458 (the AA pattern 0.525 -> 0.498 at 2048).
// 16-bit storage with one site per lane was slower blocked (FP16 step 0.280
// -> 0.289 ms); with two sites per lane (k_sweep_pairs) its particle-free
// sweep takes 199 us blocked against 211 us in planes.
constexpr int kPopBlock = 2048;
// Element of f_i at site s of a population array of q populations.
__host__ __device__ __forceinline__ int64_t pop_elem(int q, int i, int64_t s) {
  return (s / kPopBlock) * ((int64_t)q * kPopBlock) + (int64_t)i * kPopBlock + s % kPopBlock;
}
// Address of f_i at `site` (the sweep's form): the block's byte offset from
// one 32 x 32 -> 64-bit product plus a 32-bit offset within the block.
template <int Q, typename T>
__device__ __forceinline__ T* pop_at(T* p, int i, int site) {
  return (T*)((char*)p + (size_t)((uint32_t)site / kPopBlock) * (size_t)(Q * kPopBlock * sizeof(T)) +
              (uint32_t)(i * kPopBlock + (int)((uint32_t)site % kPopBlock)) * (uint32_t)sizeof(T));
}
template <int Q, typename T>
__device__ __forceinline__ const T* pop_at(const T* p, int i, int site) {
  return pop_at<Q, T>(const_cast<T*>(p), i, site);
}

// 1/rho: the hardware reciprocal in FP32 (1 ulp), a division in FP64.
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }

// Fused multiply-add in the compute type (always one rounding).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// c . v for a lattice direction (components -1, 0, 1): additions only.
template <typename Lt, typename C>
__device__ __forceinline__ C dot_c(int i, C vx, C vy, C vz) {
  C r = 0;
  if (Lt::cx(i) > 0) r += vx;
  if (Lt::cx(i) < 0) r -= vx;
  if (Lt::cy(i) > 0) r += vy;
  if (Lt::cy(i) < 0) r -= vy;
  if (Lt::cz(i) > 0) r += vz;
  if (Lt::cz(i) < 0) r -= vz;
  return r;
}

// The 16-bit collision's arithmetic, which issue rate bounds more than the
// FP32 sweep's (two sites per lane).  acc: s + v (sign > 0) or s - v into s,
// the first term taken as it is -- 0 + v costs an addition the compiler must
// keep (it is not v when v is -0); `any` is known at compile time wherever
// the direction loops are unrolled.
template <typename C>
__device__ __forceinline__ void acc(C& s, bool& any, C v, int sign) {
  if (sign > 0)
    s = any ? s + v : v;
  else
    s = any ? s - v : -v;
  any = true;
}
// c . v from the nonzero components only (0 for the rest direction).  A
// direction whose first nonzero component is negative takes minus its
// opposite's value, the same number ((-a) - b = -(a + b)), which the compiler
// then computes once per opposite pair.
template <typename Lt, typename C>
__device__ __forceinline__ C dot_c1(int i, C vx, C vy, C vz) {
  const int lead = Lt::cx(i) != 0 ? Lt::cx(i) : (Lt::cy(i) != 0 ? Lt::cy(i) : Lt::cz(i));
  const int sg = lead < 0 ? -1 : 1;
  C r = 0;
  bool any = false;
  if (Lt::cx(i) != 0) acc(r, any, vx, sg * Lt::cx(i));
  if (Lt::cy(i) != 0) acc(r, any, vy, sg * Lt::cy(i));
  if (Lt::cz(i) != 0) acc(r, any, vz, sg * Lt::cz(i));
  return sg < 0 ? -r : r;
}
// Speed class |c_i|^2 of direction i (0, 1 or 2); D2Q9 and D3Q19 weigh every
// direction of a class alike, class_w is that weight.
template <typename Lt>
__host__ __device__ constexpr int speed2(int i) {
  return Lt::cx(i) * Lt::cx(i) + Lt::cy(i) * Lt::cy(i) + Lt::cz(i) * Lt::cz(i);
}
template <int Q>
__host__ __device__ constexpr double class_w(int k) {
  for (int i = 0; i < Q; i++)
    if (speed2<Lattice<Q>>(i) == k) return Lattice<Q>::w(i);
  return 0.0;
}
// The equilibrium (eq. 2) as the 16-bit number h_i^eq = e_i / sigma at
// density deviation dr (rho = rho0 + dr) and velocity v with usq = 3/2 v.v,
// e_i = dr + rho (3 cu + 9/2 cu^2) - rho usq: the weight cancels, so it is
// kA + cu (kB + kC cu) with three constants per site, two multiply-adds per
// moving direction and none for the rest direction.
template <int Q, typename C>
struct Feq16 {
  C kA, kB, kC;
  __device__ __forceinline__ Feq16(C dr, C rho, C usq, C inv_sig) {
#pragma clang fp contract(off)
    kA = inv_sig * fmac(-rho, usq, dr);
    kB = inv_sig * C(3) * rho;
    kC = inv_sig * C(4.5) * rho;
  }
  __device__ __forceinline__ C operator()(int i, C vx, C vy, C vz) const {
#pragma clang fp contract(off)
    using L = Lattice<Q>;
    if (speed2<L>(i) == 0) return kA;
    const C cu = dot_c1<L>(i, vx, vy, vz);
    return fmac(fmac(kC, cu, kB), cu, kA);
  }
};
// Sums of 16-bit stored numbers h_i per speed class -- the weight is one per
// class, so g_i = h_i w_i sigma needs one product per class -- into the
// density deviation and momentum of the compute type D.  Each opposite pair
// (i, -i) enters as h_i + h_-i (the density) and h_i - h_-i (the momentum).
template <typename Lt>
__host__ __device__ constexpr bool lead_positive(int i) {
  return Lt::cx(i) != 0 ? Lt::cx(i) > 0 : (Lt::cy(i) != 0 ? Lt::cy(i) > 0 : Lt::cz(i) > 0);
}
template <int Q, typename T, typename D, typename C>
__device__ __forceinline__ void moments16(const C (&h)[Q], D& dr, D& jx, D& jy, D& jz) {
#pragma clang fp contract(off)
  using L = Lattice<Q>;
  D sk[3] = {0, 0, 0}, jk[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  bool hs[3] = {false, false, false};
  bool hj[3][3] = {{false, false, false}, {false, false, false}, {false, false, false}};
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int k = speed2<L>(i);
    if (k == 0) {
      acc(sk[0], hs[0], (D)h[i], 1);
      continue;
    }
    if (!lead_positive<L>(i)) continue;  // taken with its opposite
    const D a = (D)h[i], b = (D)h[opposite<Q>(i)];
    const D ps = a + b, ms = a - b;
    acc(sk[k], hs[k], ps, 1);
    if (L::cx(i) != 0) acc(jk[k][0], hj[k][0], ms, L::cx(i));
    if (L::cy(i) != 0) acc(jk[k][1], hj[k][1], ms, L::cy(i));
    if (L::cz(i) != 0) acc(jk[k][2], hj[k][2], ms, L::cz(i));
  }
  D* const out[3] = {&jx, &jy, &jz};
  bool hd = false, hm[3] = {false, false, false};
  dr = jx = jy = jz = 0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const D uk = (D)pop_unit<T>(class_w<Q>(k));
    if (hs[k]) {
      dr = hd ? fmac(uk, sk[k], dr) : uk * sk[k];
      hd = true;
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (!hj[k][a]) continue;
      *out[a] = hm[a] ? fmac(uk, jk[k][a], *out[a]) : uk * jk[k][a];
      hm[a] = true;
    }
  }
}

// Collision of one site from the populations g it pulled, in place: BGK with
// body force (eq. 1-3), the site's density deviation kept at ball sites, the
// BS substep at an owned BS site (eq. 5-7; its post-collision moments to the
// owner entry's slot) and the wall equilibrium on wall layers.  s is the
// site, fl its flag (0 without particles).  16-bit storage collides on the
// stored numbers h_i = g_i / (w_i sigma): there the weight cancels from the
// equilibrium, h_i^eq = (drho + rho (3cu + 9/2 cu^2 - 3/2 u^2)) / sigma,
// which saves the per-direction scalings; FP32/FP64 collide on the
// deviations g_i.  rec is the site's record when fl is kSiteBS (loaded by
// the caller as soon as the flag is in, so that its latency overlaps the
// population loads).  No contraction is left to the compiler (every fused
// multiply-add is written out), so every kernel that inlines this function,
// once or twice per lane, rounds every site the same way.
template <typename T>
using RecOf = decltype(ld_rec((const typename Store<T>::C*)nullptr));
template <typename T>
__device__ __forceinline__ RecOf<T> site_record(const SiteArgs<T>& sa, int s, int fl) {
  RecOf<T> r{};
  if (fl == kSiteBS) r = ld_rec(sa.vel + 4 * (size_t)s);
  return r;
}
template <int Q, typename T, bool PART>
__device__ __forceinline__ void collide_site(typename Store<T>::C (&g)[Q],
                                             const SweepArgs<Q, typename Store<T>::C>& a, const SiteArgs<T>& sa,
                                             int s, int fl, const RecOf<T>& rec, int x, int y, int z, int nx,
                                             int ny, int nz, const typename Store<T>::C (&fbt)[Q]) {
#pragma clang fp contract(off)
  using L = Lattice<Q>;
  using C = typename Store<T>::C;
  constexpr bool kRaw = std::is_same<T, _Float16>::value || std::is_same<T, bf16s>::value;
  const C inv_sig = (C)(1.0 / pop_unit<T>(1.0));
  C drho = 0, jx = 0, jy = 0, jz = 0;
  if constexpr (kRaw) {
    moments16<Q, T>(g, drho, jx, jy, jz);
  } else {
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const C v = g[i];
      drho += v;
      if (L::cx(i) > 0) jx += v;
      if (L::cx(i) < 0) jx -= v;
      if (L::cy(i) > 0) jy += v;
      if (L::cy(i) < 0) jy -= v;
      if (L::cz(i) > 0) jz += v;
      if (L::cz(i) < 0) jz -= v;
    }
  }
  const C rho = a.rho0 + drho;
  const C inv = recip(rho);
  const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const C usq = C(1.5) * fmac(ux, ux, fmac(uy, uy, uz * uz));
  if constexpr (kRaw) {
    const Feq16<Q, C> fe(drho, rho, usq, inv_sig);
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const C r = fmac(a.omega, fe(i, ux, uy, uz) - g[i], g[i]);
      // the body-force term 3 w_i c_i . f_b, in stored units (0 at rest)
      g[i] = speed2<L>(i) == 0 ? r : fmac(fbt[i], (C)(1.0 / pop_unit<T>(L::w(i))), r);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const C cu = dot_c<L>(i, ux, uy, uz);
      const C geq = C(L::w(i)) * fmac(rho, fmac(C(4.5) * cu, cu, fmac(C(3), cu, -usq)), drho);
      g[i] = fmac(a.omega, geq - g[i], g[i]) + fbt[i];
    }
  }
  if (PART && fl != 0) {
    sa.drho[s] = drho;
    if (fl == kSiteBS) {
      // BS substep at an owned BS site: its post-collision moments go to the
      // owner's slot (FP64 sums), and the populations become f^eq(rho_B,
      // u_B') with the rigid-body velocity u_B' = u_p + omega x r of the site
      const C vx = rec.x, vy = rec.y, vz = rec.z;
      const int bs = as_idx<C>(rec.w);
      double dr = 0, bx = 0, by = 0, bz = 0;
      if constexpr (kRaw) {
        moments16<Q, T>(g, dr, bx, by, bz);
      } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          const double v = (double)g[i];
          dr += v;
          if (L::cx(i) > 0) bx += v;
          if (L::cx(i) < 0) bx -= v;
          if (L::cy(i) > 0) by += v;
          if (L::cy(i) < 0) by -= v;
          if (L::cz(i) > 0) bz += v;
          if (L::cz(i) < 0) bz -= v;
        }
      }
      if ((unsigned)bs < (unsigned)sa.nent) {
        double* sl = sa.slot + 4 * (size_t)bs;
        sl[0] = dr;
        sl[1] = bx;
        sl[2] = by;
        sl[3] = bz;
      } else {
        // a record that names no entry (never written by the prepare pass):
        // no write through it; the next synchronising call reports it
        atomicOr(sa.status, kStatusRecord);
      }
      const C drB = (C)dr;
      const C rhoB = a.rho0 + drB;
      const C usqB = C(1.5) * fmac(vx, vx, fmac(vy, vy, vz * vz));
      if constexpr (kRaw) {
        const Feq16<Q, C> fe(drB, rhoB, usqB, inv_sig);
#pragma unroll
        for (int i = 0; i < Q; i++) g[i] = fe(i, vx, vy, vz);
      } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          const C cu = dot_c<L>(i, vx, vy, vz);
          g[i] = C(L::w(i)) * fmac(rhoB, fmac(C(4.5) * cu, cu, fmac(C(3), cu, -usqB)), drB);
        }
      }
    }
  }
  if (a.walls) {
    // wall layers: f^eq(rho, U_wall) with the site's own density (no
    // particle owns a wall site, so no BS exchange above touched it)
    C vx, vy, vz;
    if (wall_velocity(a, x, y, z, nx, ny, nz, vx, vy, vz)) {
      const C usqW = C(1.5) * fmac(vx, vx, fmac(vy, vy, vz * vz));
      if constexpr (kRaw) {
        const Feq16<Q, C> fe(drho, rho, usqW, inv_sig);
#pragma unroll
        for (int i = 0; i < Q; i++) g[i] = fe(i, vx, vy, vz);
      } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          const C cu = dot_c<L>(i, vx, vy, vz);
          g[i] = C(L::w(i)) * fmac(rho, fmac(C(4.5) * cu, cu, fmac(C(3), cu, -usqW)), drho);
        }
      }
    }
  }
}

// The work of one site (x, y, z) of a box of nx x ny x nz sites whose first
// site is `off`; fbt holds 3 w_i c_i . f_b of that box.  NTL: streaming
// (non-temporal) population loads.  Each pulled value is read once, so on
// long rows they only keep dead lines out of the caches; in an ensemble of
// narrow boxes the lines shared by neighbouring tiles are worth keeping.
template <int Q, typename T, bool PART, int LAY, bool NTL>
__device__ __forceinline__ void sweep_site(const T* A, T* B, const SweepArgs<Q, typename Store<T>::C>& a,
                                           const SiteArgs<T>& sa, int x, int y, int z, int nx, int ny, int nz,
                                           int off, const typename Store<T>::C (&fbt)[Q]) {
  using L = Lattice<Q>;
  using C = typename Store<T>::C;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const int s = off + x + nx * (y + ny * z);

  // the flag is issued first and waited on only after the collision
  const int fl = PART ? (int)sa.flag[s] : 0;
  constexpr bool kRaw = std::is_same<T, _Float16>::value || std::is_same<T, bf16s>::value;
  // Addresses: the block's byte offset from one 32 x 32 -> 64-bit product and
  // a 32-bit offset within the block (pop_at).
  C g[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    // f_i arriving at x: pulled from x - c_i, or found at x itself in the
    // post-propagation half of the AA pattern
    const int sx = LAY == kLayAAStream ? x : (L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x));
    const int sy = LAY == kLayAAStream ? y : (L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y));
    const int sz = LAY == kLayAAStream ? z : (L::cz(i) > 0 ? zm : (L::cz(i) < 0 ? zp : z));
    const T* src = pop_at<Q, T>(A, LAY == kLayAASwap ? opposite<Q>(i) : i, off + sx + nx * (sy + ny * sz));
    const C h = NTL ? Store<T>::ldnt(src) : Store<T>::ld(src);
    g[i] = kRaw ? h : h * (C)pop_unit<T>(L::w(i));
  }
  const RecOf<T> rec = PART ? site_record(sa, s, fl) : RecOf<T>{};
  collide_site<Q, T, PART>(g, a, sa, s, fl, rec, x, y, z, nx, ny, nz, fbt);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    // f*_i(x): at x in the next array, in the opposite slot at x, or pushed to
    // x + c_i (the three layouts above)
    const int dx = LAY == kLayAASwap ? (L::cx(i) > 0 ? xp : (L::cx(i) < 0 ? xm : x)) : x;
    const int dy = LAY == kLayAASwap ? (L::cy(i) > 0 ? yp : (L::cy(i) < 0 ? ym : y)) : y;
    const int dz = LAY == kLayAASwap ? (L::cz(i) > 0 ? zp : (L::cz(i) < 0 ? zm : z)) : z;
    T* dst = pop_at<Q, T>(B, LAY == kLayAAStream ? opposite<Q>(i) : i, off + dx + nx * (dy + ny * dz));
    if constexpr (kRaw)
      Store<T>::st(dst, g[i]);
    else
      pop_st<Q, T>(dst, i, g[i]);
  }
}

// One box: workgroup (bx, y, z) covers kSweepBlock sites of row (y, z), with
// streaming loads.
template <int Q, typename T, bool PART, int LAY>
__global__ __launch_bounds__(kSweepBlock) void k_sweep(const T* A, T* B, SweepArgs<Q, typename Store<T>::C> a,
                                                        SiteArgs<T> sa) {
  const int x = (int)blockIdx.x * kSweepBlock + (int)threadIdx.x;
  if (x >= a.nx) return;
  sweep_site<Q, T, PART, LAY, true>(A, B, a, sa, x, (int)blockIdx.y, (int)blockIdx.z, a.nx, a.ny, a.nz, 0, a.fbt);
}

// 16-bit storage, two arrays, nx even: two sites per lane.  A wave takes 128
// consecutive sites of a row (64 site pairs, x even), so each population is
// one aligned 4-byte load per lane, 256 bytes per wave as FP32 moves with one
// site per lane (2-byte loads of one site per lane stream about 10 % slower).
// The pull's shift by one site along x (populations with c_x != 0) is rebuilt
// from the neighbouring lane's word (DPP wave shift by one lane) and, at the
// wave's two ends, from the word past the end: the last word of the wave
// before it in the row (periodic) or the first word of the one after it.
// Those waves load these words for themselves; when they belong to the same
// workgroup (every wave of the 256^3 box: two rows of two waves) the words
// are passed through LDS, otherwise loaded once more with a wave-uniform
// load (such loads missed the caches and fetched a line from HBM each).
// Each site collides as in sweep_site (collide_site), so the results are the
// same bits.  Lanes past the row's end repeat its last pair and store
// nothing; waves past the last row repeat it and store nothing, so that
// every wave of the workgroup meets its barrier.
template <typename T>
__device__ __forceinline__ float half_lo(uint32_t v) {
  if constexpr (std::is_same<T, _Float16>::value)
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
  else
    return bf16_bits_to_f32((uint16_t)(v & 0xffffu));
}
// Two compute-type values rounded to the storage type (nearest even) and
// packed, lo in the low half: one conversion instruction for both.
template <typename T>
__device__ __forceinline__ uint32_t pack_halves(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 v = {lo, hi};
  if constexpr (std::is_same<T, _Float16>::value) {
    typedef _Float16 t2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, t2));
  } else {
    typedef __bf16 t2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, t2));
  }
}
constexpr int kPairRow = 128;  // sites of a row per wave of k_sweep_pairs
// Index of population i among those with c_x != 0 (and their count, i = Q).
template <typename Lt>
__host__ __device__ constexpr int x_shifted_before(int i) {
  int n = 0;
  for (int k = 0; k < i; k++) n += Lt::cx(k) != 0;
  return n;
}

template <int Q, typename T, bool PART>
__global__ __launch_bounds__(kSweepBlock) void k_sweep_pairs(const T* __restrict__ A, T* __restrict__ B,
                                                              SweepArgs<Q, float> a, SiteArgs<T> sa) {
  static_assert(sizeof(T) == 2, "two sites per lane: 16-bit storage");
  using L = Lattice<Q>;
  constexpr int kWaves = kSweepBlock / 64;
  constexpr int kShift = x_shifted_before<L>(Q);
  __shared__ uint32_t s_edge[kWaves][2][kShift];  // [wave][first, last word][shifted population]
  const int lane = (int)threadIdx.x & 63;
  // wave-uniform: the row chunk of this wave (the last one for waves past it)
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int cpr = (nx + kPairRow - 1) / kPairRow;
  const int items = cpr * ny * nz;
  const int w0 = (int)blockIdx.x * kWaves;
  const bool live = w0 + wv < items;
  const int item = live ? w0 + wv : items - 1;
  const int row = item / cpr, chunk = item - row * cpr, xw = chunk * kPairRow;
  const int y = row % ny, z = row / ny;
  const int npair = min(kPairRow / 2, (nx - xw) / 2);
  const bool act = live && lane < npair;
  const int x = xw + 2 * min(lane, npair - 1);
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const int s = x + nx * (y + ny * z);
  // the pair's two flag bytes (s even: one aligned 2-byte load)
  const int fl2 = PART ? (int)*(const uint16_t*)(sa.flag + s) : 0;
  // the waves before and after this one along the row (periodic), and
  // whether this workgroup holds them; otherwise the word past the end is
  // loaded here: sites (xl, xl + 1) hold x - 1 of the first site, (xr, xr + 1)
  // x + 1 of the last
  const int left = chunk == 0 ? item + cpr - 1 : item - 1;
  const int right = chunk == cpr - 1 ? item - (cpr - 1) : item + 1;
  const bool left_here = live && left >= w0 && left < w0 + kWaves;
  const bool right_here = live && right >= w0 && right < w0 + kWaves;
  const int xl = xw == 0 ? nx - 2 : xw - 2;
  const int xr = xw + 2 * npair == nx ? 0 : xw + 2 * npair;
  uint32_t d[Q], e[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y);
    const int sz = L::cz(i) > 0 ? zm : (L::cz(i) < 0 ? zp : z);
    const int rs = nx * (sy + ny * sz);
    d[i] = __builtin_nontemporal_load((const uint32_t*)pop_at<Q, T>(A, i, rs + x));
    e[i] = 0;
    if (L::cx(i) > 0 && !left_here) e[i] = *(const uint32_t*)pop_at<Q, T>(A, i, rs + xl);
    if (L::cx(i) < 0 && !right_here) e[i] = *(const uint32_t*)pop_at<Q, T>(A, i, rs + xr);
  }
  // the records of owned BS sites, issued before the populations are waited on
  const int fa = act ? fl2 & 0xff : 0, fb = act ? fl2 >> 8 : 0;
  const RecOf<T> ra = PART ? site_record(sa, s, fa) : RecOf<T>{};
  const RecOf<T> rb = PART ? site_record(sa, s + 1, fb) : RecOf<T>{};
  // pass the first and last words of the shifted populations to the
  // neighbouring waves of this workgroup
#pragma unroll
  for (int i = 0; i < Q; i++) {
    if (L::cx(i) == 0) continue;
    const int k = x_shifted_before<L>(i);
    if (lane == 0) s_edge[wv][0][k] = d[i];
    if (lane == npair - 1) s_edge[wv][1][k] = d[i];
  }
  __syncthreads();
  float ga[Q], gb[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    uint32_t v = d[i];
    const int k = x_shifted_before<L>(i);
    if (L::cx(i) > 0) {  // from x - 1: the high half of the previous word, the low half of this one
      uint32_t p = __builtin_amdgcn_update_dpp(0u, d[i], 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
      if (lane == 0) p = left_here ? s_edge[left - w0][1][k] : e[i];
      v = __builtin_amdgcn_alignbit(d[i], p, 16);
    } else if (L::cx(i) < 0) {  // from x + 1: the high half of this word, the low half of the next one
      uint32_t n = __builtin_amdgcn_update_dpp(0u, d[i], 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
      if (lane == npair - 1) n = right_here ? s_edge[right - w0][0][k] : e[i];
      v = __builtin_amdgcn_alignbit(n, d[i], 16);
    }
    ga[i] = half_lo<T>(v);
    gb[i] = half_lo<T>(v >> 16);
  }
  collide_site<Q, T, PART>(ga, a, sa, s, fa, ra, x, y, z, nx, ny, nz, a.fbt);
  collide_site<Q, T, PART>(gb, a, sa, s + 1, fb, rb, x + 1, y, z, nx, ny, nz, a.fbt);
  if (act) {
#pragma unroll
    for (int i = 0; i < Q; i++)
      __builtin_nontemporal_store(pack_halves<T>(ga[i], gb[i]), (uint32_t*)pop_at<Q, T>(B, i, s));
  }
}

// q = n / d for 0 <= n < 2^31, 1 <= d, from inv = 1/d rounded to FP64: the
// product is within 2^-21 of n/d, so truncation is off by at most one and the
// remainder corrects it.
__device__ __forceinline__ int div_exact(int n, int d, double inv) {
  const int q = (int)((double)n * inv);
  const int64_t r = (int64_t)n - (int64_t)q * d;
  return q + (r >= d) - (r < 0);
}

// Any number of boxes: a tile is up to blockDim.x consecutive sites of one
// box in raster order (x fastest, running on into the next row), starting at
// a multiple of blockDim.x of the whole site range (a box's first tile may be
// shorter), so the tile's accesses are contiguous whatever the box width and
// its stores fill whole lines.  Three records per tile: {box, first box-local
// site, one past its last, -}, the box's {nx, ny, nz, first site}, and 1/nx,
// 1/ny as FP64 bit pairs {lo, hi, lo, hi} for the split of a box-local index
// into (x, y, z).  A persistent grid walks the tile list (the workgroup
// width, grid size and occupancy cap are the tunable launch shape).
template <int Q, typename T, bool PART, int LAY, bool NTL>
__global__ __launch_bounds__(kTileMax) void k_sweep_tiles(const T* A, T* B, SweepArgs<Q, typename Store<T>::C> a,
                                                           SiteArgs<T> sa,
                                                           const int4* __restrict__ tiles, int ntiles,
                                                           const typename Store<T>::C* __restrict__ fbt_tab) {
  using C = typename Store<T>::C;
  // An ensemble's tiles share the lines at their ends (a tile pulls runs of
  // its sites shifted by c_x + n_x c_y), so with one workgroup per tile
  // (grid 0) runs of kXcdRun adjacent tiles go to one XCD: workgroups are
  // dealt to the eight XCDs in turn, and the shared lines then meet in one
  // L2 (64-box D2Q9 ensemble: 0.1517 -> 0.1495 ms per step tuned, +6.5 %
  // MLUPS eager).  One box keeps the hardware's order (its tiles are whole
  // rows that share no lines, and the regrouped order was 0.3 % slower).
  int t0 = blockIdx.x;
  if (!NTL && (int)gridDim.x == ntiles) {
    constexpr int R = 8 * kXcdRun;
    if (t0 < ntiles / R * R) t0 = t0 / R * R + kXcdRun * (t0 % 8) + (t0 / 8) % kXcdRun;
  }
  for (int t = t0; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[3 * t], tg = tiles[3 * t + 1], ti = tiles[3 * t + 2];
    const int64_t lin64 = (int64_t)tl.y + threadIdx.x;
    if (lin64 >= tl.z) continue;  // past the tile's last site
    const int lin = (int)lin64;
    const int yz = div_exact(lin, tg.x, __hiloint2double(ti.y, ti.x));
    const int z = div_exact(yz, tg.y, __hiloint2double(ti.w, ti.z));
    C fb[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) fb[i] = fbt_tab[tl.x * Q + i];
    sweep_site<Q, T, PART, LAY, NTL>(A, B, a, sa, lin - yz * tg.x, yz - z * tg.y, z, tg.x, tg.y, tg.z, tg.w, fb);
  }
}

// ---------------------------------------------------------------------------
// Deterministic sums: butterfly within the 64-wide wave, then waves in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Exclusive prefix sum of c over a workgroup of NT threads: a shuffle scan in
// each wave, then the wave totals (s_w holds NT/64 ints).  Returns this
// thread's offset; total receives the workgroup's sum.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int c, int* s_w, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int v = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == 63) s_w[wv] = v;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; w++) {
    const int t = s_w[w];
    before += w < wv ? t : 0;
    tot += t;
  }
  __syncthreads();  // s_w is free again
  total = tot;
  return before + v - c;
}

// ---------------------------------------------------------------------------
// K3: particle update (eq. 10-11, 16-19, 13), one workgroup per box: boxes
// are independent, and a box's particles have consecutive ids p0 .. p1-1.
// Positions, velocities, masses and radii of a box of up to kStageParticles
// particles are staged in LDS, and the box's candidate pairs are compacted in
// lexicographic order (each particle's list is in increasing j); one thread
// then walks the pairs -- each collision acts on the velocities earlier ones
// left -- against LDS instead of a chain of dependent memory loads.
// ---------------------------------------------------------------------------
constexpr int kStageParticles = 640;  // particles of one box staged in LDS
constexpr int kStagePairs = 2048;     // candidate pairs of one box staged in LDS (the rest in memory)

// A box's particle state, staged ([component][particle - p0]) or in the
// particle arrays ([particle][component]).
struct PartView {
  double* x;
  double* u;
  const double* m;
  const double* r;
  int sa, sp, p0;
  __device__ __forceinline__ double& X(int p, int a) const { return x[a * sa + (p - p0) * sp]; }
  __device__ __forceinline__ double& U(int p, int a) const { return u[a * sa + (p - p0) * sp]; }
  __device__ __forceinline__ double M(int p) const { return m[p - p0]; }
  __device__ __forceinline__ double R(int p) const { return r[p - p0]; }
};

template <int NT>
__global__ __launch_bounds__(NT) void k_particles(DevParticles P, int dim, Boxes BX, int* status) {
  __shared__ double s_x[3 * kStageParticles], s_u[3 * kStageParticles], s_m[kStageParticles], s_r[kStageParticles];
  __shared__ int2 s_pairs[kStagePairs];
  __shared__ int s_scan[NT / 64];
  __shared__ double s_vmax[NT / 64];
  const int b = blockIdx.x;
  const Geo G = BX.nbox == 1 ? BX.g0 : BX.tab[b];
  const int p0 = b == 0 ? 0 : BX.tab[b - 1].p1, p1 = G.p1;
  if (p1 <= p0) return;  // an empty box (uniform over the workgroup)
  const bool staged = p1 - p0 <= kStageParticles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int L[3] = {G.nx, G.ny, G.nz};
  double vmax = 0;
  // one particle per thread: the translation's inputs and the candidate
  // count are loaded with the first phase's, not after the pair pass
  const bool one = p1 - p0 <= NT;
  double xr[3] = {0, 0, 0}, x0r[3] = {0, 0, 0};
  int k0r[3] = {0, 0, 0}, b0r[3] = {0, 0, 0}, ogr[3] = {0, 0, 0};
  int cnr = 0;
  for (int p = p0 + tid; p < p1; p += NT) {
    // every input is loaded before the first store: the particle arrays
    // could alias as far as the compiler knows, and a load after a store
    // would wait for it
    const double m = P.m[p], I = P.I[p], rad = P.rad[p];
    double dp[3], dl[3], fc[3], u[3], fe[3], om[3], x[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      dp[a] = P.dP[3 * p + a];
      dl[a] = P.dL[3 * p + a];
      fc[a] = P.fc[3 * p + a];
      u[a] = P.u[3 * p + a];
      fe[a] = P.fext[3 * p + a];
      om[a] = P.om[3 * p + a];
      x[a] = P.x[3 * p + a];
    }
    if (one) {
#pragma unroll
      for (int a = 0; a < 3; a++) {
        x0r[a] = P.x0[3 * p + a];
        k0r[a] = P.k[3 * p + a];
        b0r[a] = P.b0[3 * p + a];
        ogr[a] = P.org[3 * p + a];
        xr[a] = x[a];
      }
      cnr = P.cand_n[p];
    }
    double v2 = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (!isinf(m)) u[a] = u[a] + (fe[a] - dp[a] + fc[a]) / m;
      if (!isinf(I)) om[a] = om[a] - dl[a] / I;
      v2 += u[a] * u[a];
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
      P.F[3 * p + a] = -dp[a] + fc[a];
      P.T[3 * p + a] = -dl[a];
      P.u[3 * p + a] = u[a];
      P.om[3 * p + a] = om[a];
      if (staged) {
        s_x[a * kStageParticles + p - p0] = x[a];
        s_u[a * kStageParticles + p - p0] = u[a];
      }
    }
    if (staged) {
      s_m[p - p0] = m;
      s_r[p - p0] = rad;
    }
    vmax = fmax(vmax, sqrt(v2));
  }
  for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  if (lane == 0) s_vmax[wv] = vmax;

  // the box's candidate pairs in lexicographic order: the first kStagePairs
  // in LDS, any others in the box's part of the pair buffer (a particle has
  // at most kCandMax candidates, so the part holds them all)
  int2* gpairs = (int2*)P.pairs + (size_t)p0 * kCandMax;
  int total = 0;
  for (int c0 = p0; c0 < p1; c0 += NT) {
    const int p = c0 + tid;
    const int c = p < p1 ? (one ? cnr : P.cand_n[p]) : 0;
    int chunk;
    const int excl = total + block_excl_scan<NT>(c, s_scan, chunk);
    for (int t = 0; t < c; t++) {
      const int k = excl + t;
      const int2 pr = make_int2(p, P.cand[p * kCandMax + t]);
      if (k < kStagePairs)
        s_pairs[k] = pr;
      else
        gpairs[k] = pr;
    }
    total += chunk;
  }
  __syncthreads();

  double vseen = 0;
  if (tid == 0) {
    const PartView V = staged ? PartView{s_x, s_u, s_m, s_r, kStageParticles, 1, p0}
                              : PartView{P.x, P.u, P.m, P.rad, 1, 3, 0};
    for (int k = 0; k < total; k++) {
      const int2 pr = k < kStagePairs ? s_pairs[k] : gpairs[k];
      const int i = pr.x, j = pr.y;
      const double mi = V.M(i), mj = V.M(j), ri = V.R(i), rj = V.R(j);
      const bool infA = isinf(mi), infB = isinf(mj);
      if (infA && infB) continue;
      double d[3], dd = 0;
      for (int a = 0; a < 3; a++) {
        d[a] = (V.X(j, a) + V.U(j, a)) - (V.X(i, a) + V.U(i, a));
        if (a < dim) d[a] = d[a] - L[a] * floor(d[a] / L[a] + 0.5);
        dd += d[a] * d[a];
      }
      const double dist = sqrt(dd);
      if (dist > ri + rj || dist == 0.0) continue;
      double n[3], vn = 0;
      for (int a = 0; a < 3; a++) {
        n[a] = d[a] / dist;
        vn += (V.U(j, a) - V.U(i, a)) * n[a];
      }
      if (!(vn < 0.0)) continue;
      double W[3];
      for (int a = 0; a < 3; a++) {
        if (infA)
          W[a] = V.U(i, a);
        else if (infB)
          W[a] = V.U(j, a);
        else
          W[a] = (mi * V.U(i, a) + mj * V.U(j, a)) / (mi + mj);
      }
      const int who[2] = {i, j};
      for (int t2 = 0; t2 < 2; t2++) {
        const int q = who[t2];
        double wvv[3], wn = 0, v2 = 0;
        for (int a = 0; a < 3; a++) {
          wvv[a] = V.U(q, a) - W[a];
          wn += wvv[a] * n[a];
        }
        for (int a = 0; a < 3; a++) {
          const double u = W[a] + (wvv[a] - 2.0 * wn * n[a]);
          V.U(q, a) = u;
          v2 += u * u;
        }
        vseen = fmax(vseen, sqrt(v2));
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double vm = vseen;
    for (int w = 0; w < NT / 64; w++) vm = fmax(vm, s_vmax[w]);
    if (2.0 * vm >= kMargin) atomicOr(status, kStatusCollision);
  }
  for (int p = p0 + tid; p < p1; p += NT) {
    // inputs first, as above
    const double m = P.m[p], r = P.rad[p];
    double u[3], x[3], x0[3];
    int k0[3], b0[3], og[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      u[a] = staged ? s_u[a * kStageParticles + p - p0] : P.u[3 * p + a];
      x[a] = one ? xr[a] : P.x[3 * p + a];
      x0[a] = one ? x0r[a] : P.x0[3 * p + a];
      k0[a] = one ? k0r[a] : P.k[3 * p + a];
      b0[a] = one ? b0r[a] : P.b0[3 * p + a];
      og[a] = one ? ogr[a] : P.org[3 * p + a];
    }
    if (G.walls && !isinf(m)) {
      // contact with a wall after the pairs: the normal velocity reverses
      // when the predicted surface reaches the BS layer while approaching
      for (int a = 0; a < dim; a++) {
        if (!(G.walls & (1 << a))) continue;
        const double xp = x[a] + u[a];
        if ((xp - r <= 1.0 && u[a] < 0.0) || (xp + r >= (double)(L[a] - 2) && u[a] > 0.0)) u[a] = -u[a];
      }
    }
    int moved = 0;
    for (int a = 0; a < 3; a++) {
      P.u[3 * p + a] = u[a];
      P.orgp[3 * p + a] = og[a];  // the site sets before this translation
    }
    for (int a = 0; a < dim; a++) {
      const double xn = x[a] + u[a];
      P.x[3 * p + a] = xn;
      const int k = (int)floor(xn - x0[a] + 0.5);
      moved += k != k0[a];
      P.k[3 * p + a] = k;
      P.org[3 * p + a] = wrap(b0[a] + k, L[a]);
    }
    // a shift along all three axes at once (not a D3Q19 link) can take an IS
    // site outside the ball the sweep kept densities for
    P.jump[p] = moved == 3;
    P.moved[p] = moved != 0;
  }
}

// ---------------------------------------------------------------------------
// K2: per-particle sums of the BS slots (eq. 8-9) in a fixed order, release
// of the particle's stamps, and the list of particles close enough to collide
// this step.  One workgroup per particle.
// ---------------------------------------------------------------------------
// GRID: site ownership is settled from kind grids after the particle update,
// so the map and flags are not released here, and the particles that may
// share a site with this one (both directions) are listed for it; otherwise
// every claim and flag of the particle is released at its current shift.
template <int NB, bool GRID>
__global__ __launch_bounds__(NB) void k_reduce(int* __restrict__ own,
                                                            uint8_t* __restrict__ flag, const double* __restrict__ slot,
                                                            DevParticles P, DevEntries E, Boxes BX,
                                                            double rho0, double margin, int* status) {
  constexpr int kWaves = NB / 64;
  __shared__ double s_part[kWaves][6];
  __shared__ int s_cnt[kWaves], s_cnt2[kWaves];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const Geo G = geo_of(BX, P, p);
  const int e0 = P.ent0[p], nbs = P.nbs[p], nis = P.nis[p], nin = P.nin[p];
  const double phx = P.phi[3 * p], phy = P.phi[3 * p + 1], phz = P.phi[3 * p + 2];
  const double upx = P.u[3 * p], upy = P.u[3 * p + 1], upz = P.u[3 * p + 2];
  const double wx = P.om[3 * p], wy = P.om[3 * p + 1], wz = P.om[3 * p + 2];
  // the wrapped origin, loaded once (a load inside the entry loop would wait
  // for the map stores before it, which the compiler cannot prove distinct)
  const int ox0 = P.org[3 * p], oy0 = P.org[3 * p + 1], oz0 = P.org[3 * p + 2];

  // Close neighbours j > p in the same box (positions before translation):
  // the first chunk's test is issued here, so that its loads overlap the
  // entry loads below; the list is built after the sums.
  const double xpx = P.x[3 * p], xpy = P.x[3 * p + 1], xpz = P.x[3 * p + 2];
  const double rp = P.rad[p];
  const int np = G.p1;
  // squared minimum-image distance to (xj, yj, zj)
  auto dist2 = [&](double xj, double yj, double zj) {
    double dx = xj - xpx, dy = yj - xpy, dz = zj - xpz;
    dx -= G.nx * floor(dx / G.nx + 0.5);
    dy -= G.ny * floor(dy / G.ny + 0.5);
    if (G.nz > 1) dz -= G.nz * floor(dz / G.nz + 0.5);
    return dx * dx + dy * dy + dz * dz;
  };
  // the scan runs over j > p, or over the whole box for the site-sharing list
  const int bq = BX.nbox == 1 ? 0 : P.box[p];
  const int jstart = GRID ? (bq == 0 ? 0 : BX.tab[bq - 1].p1) : p + 1;
  // the first chunk's positions, loaded without a branch (lanes past the box's
  // last particle load this particle's own) and tested after the sums
  const int j1 = jstart + tid;
  const int jc = j1 < np ? j1 : p;
  const double xj1 = P.x[3 * jc], yj1 = P.x[3 * jc + 1], zj1 = P.x[3 * jc + 2], rj1 = P.rad[jc];

  double acc[6] = {0, 0, 0, 0, 0, 0};
  // the sums need the BS entries (the first nbs of the particle); releasing
  // the map and flags (owner-map mode) needs every entry
  const int ne = GRID ? nbs : nbs + nis + nin;
  constexpr int kEnt = 4;  // entries per thread whose loads are issued together
  for (int tb = 0; tb < ne; tb += NB * kEnt) {
    // every entry's offset and slot, loaded together and without per-lane
    // branches (lanes past the last entry load the last one again and drop
    // it): only the slots of BS entries hold moments (or the unowned mark)
    int pkv[kEnt];
    double4 mv[kEnt];
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if (tb + j * NB >= ne) break;  // the same for the whole workgroup
      const int e = e0 + min(tb + j * NB + tid, ne - 1);
      pkv[j] = E.off[e];
      mv[j] = *(const double4*)(slot + 4 * (size_t)e);
    }
    // the sums first, the stores after: a wait for a loaded value placed
    // between two stores would also wait for the first store (the vector
    // memory counter counts both)
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if (tb + j * NB >= ne) break;
      const int t = tb + j * NB + tid;
      const int pk = pkv[j];
      if (t >= ne || entry_kind(pk) != 1 || mv[j].x == kSlotUnowned) continue;  // owned BS sites only
      // dp = rho_B (u_B' - u_B), dl = r x dp with the post-collision moments
      const double rhoB = rho0 + mv[j].x;
      const double ubx = mv[j].y / rhoB, uby = mv[j].z / rhoB, ubz = mv[j].w / rhoB;
      const double rx = (double)off_x(pk) - phx, ry = (double)off_y(pk) - phy, rz = (double)off_z(pk) - phz;
      const double vx = upx + (wy * rz - wz * ry);
      const double vy = upy + (wz * rx - wx * rz);
      const double vz = upz + (wx * ry - wy * rx);
      const double dpx = rhoB * (vx - ubx), dpy = rhoB * (vy - uby), dpz = rhoB * (vz - ubz);
      acc[0] += dpx;
      acc[1] += dpy;
      acc[2] += dpz;
      acc[3] += ry * dpz - rz * dpy;
      acc[4] += rz * dpx - rx * dpz;
      acc[5] += rx * dpy - ry * dpx;
    }
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if (tb + j * NB >= ne) break;
      const int t = tb + j * NB + tid;
      if (t >= ne) continue;
      const int pk = pkv[j];
      if constexpr (!GRID) {
        const int s = site_of(G, wrap1(ox0 + off_x(pk), G.nx), wrap1(oy0 + off_y(pk), G.ny),
                              wrap1(oz0 + off_z(pk), G.nz));
        flag[s] = 0;
        // every claim at s is released this step, the owner's among them, so
        // each BS/IS entry clears s without asking whose it is
        if (entry_kind(pk) != 3) own[s] = kEmpty;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; c++) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) s_part[wv][c] = v;
  }
  __syncthreads();
  if (tid < 6) {
    double v = 0;
    for (int w = 0; w < kWaves; w++) v += s_part[w][tid];
    if (tid < 3)
      P.dP[3 * p + tid] = v;
    else
      P.dL[3 * p + tid - 3] = v;
  }

  // The close neighbours listed in increasing j: the only pairs that can pass
  // the collision test this step while every speed stays below kMargin / 2
  // (checked in the particle update), and, with margin >= the closure's gap,
  // every pair the closure acts on.
  // With GRID, the same scan lists in increasing j every other particle of
  // the box within r_p + r_j + kShareMargin: those whose sites may coincide
  // with this particle's after the translation of this step.
  int base = 0, nbase = 0;
  for (int j0 = jstart; j0 < np; j0 += NB) {
    const int j = j0 + tid;
    const int jj = j < np ? j : p;
    double xj = xj1, yj = yj1, zj = zj1, rj = rj1;
    if (j0 != jstart) {
      xj = P.x[3 * jj];
      yj = P.x[3 * jj + 1];
      zj = P.x[3 * jj + 2];
      rj = P.rad[jj];
    }
    const double d2 = dist2(xj, yj, zj);
    const double lim = rp + rj + margin, lims = rp + rj + kShareMargin;
    const bool close = j < np && j > p && d2 <= lim * lim;
    const bool share = GRID && j < np && j != p && d2 <= lims * lims;
    const unsigned long long bal = __ballot(close);
    const unsigned long long bal2 = __ballot(share);
    if (lane == 0) {
      s_cnt[wv] = __popcll(bal);
      s_cnt2[wv] = __popcll(bal2);
    }
    __syncthreads();
    int off = base, off2 = nbase;
    int tot = 0, tot2 = 0;
    for (int w = 0; w < kWaves; w++) {
      if (w < wv) {
        off += s_cnt[w];
        off2 += s_cnt2[w];
      }
      tot += s_cnt[w];
      tot2 += s_cnt2[w];
    }
    if (close) {
      const int idx = off + __popcll(bal & ((1ull << lane) - 1ull));
      if (idx < kCandMax) P.cand[p * kCandMax + idx] = j;
    }
    if (share) {
      const int idx = off2 + __popcll(bal2 & ((1ull << lane) - 1ull));
      if (idx < kNbrMax) P.nbr[(size_t)p * kNbrMax + idx] = j;
    }
    base += tot;
    nbase += tot2;
    __syncthreads();
  }
  if (tid == 0) {
    P.cand_n[p] = base < kCandMax ? base : kCandMax;
    if (GRID) P.nbr_n[p] = nbase < kNbrMax ? nbase : kNbrMax;
    if (base > kCandMax || (GRID && nbase > kNbrMax)) atomicOr(status, kStatusCollision);
  }

}

// ---------------------------------------------------------------------------
// K4: stamp every template entry at its particle's shift: BS/IS entries
// claim the owner map (lowest index, hence lowest particle id, wins).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stamp(int* __restrict__ own, DevParticles P,
                                                DevEntries E, Boxes BX, int e_begin, int e_end) {
  const int e = e_begin + blockIdx.x * 256 + threadIdx.x;
  if (e >= e_end) return;
  const int pk = E.off[e];
  const int p = E.pid[e];
  const Geo G = geo_of(BX, P, p);
  int x, y, z;
  entry_xyz(P, G, p, pk, x, y, z);
  const int s = site_of(G, x, y, z);
  const int kind = entry_kind(pk);
  // wall sites belong to the wall
  if (kind != 3 && !wall_site(G, x, y, z)) atomicMin(&own[s], 2 * e + (kind == 2));
}

// The same for every particle, one workgroup each: the particle's box, origin
// and entry range are uniform loads and its entries coalesced ones, so each
// entry costs one dependent load before its stores (the per-step stamp).
__global__ __launch_bounds__(256) void k_stamp_particles(int* __restrict__ own, DevParticles P, DevEntries E,
                                                         Boxes BX, int split) {
  // split workgroups per particle, rows of 256 entries dealt round-robin
  const int p = blockIdx.x / split, part = blockIdx.x % split;
  const Geo G = geo_of(BX, P, p);
  const int e0 = P.ent0[p], ne = P.nbs[p] + P.nis[p] + P.nin[p];
  const int ox = P.org[3 * p], oy = P.org[3 * p + 1], oz = P.org[3 * p + 2];
  // the offsets of kEnt entries per thread are loaded before any of their
  // atomics, which the compiler would otherwise keep in order with the loads
  constexpr int kEnt = 4;
  for (int rb = part; rb * 256 < ne; rb += split * kEnt) {
    int pkv[kEnt];
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if ((rb + j * split) * 256 >= ne) break;  // the same for the whole workgroup
      pkv[j] = E.off[e0 + min((rb + j * split) * 256 + (int)threadIdx.x, ne - 1)];
    }
    // every site and code first, the atomics after, back to back (a wait for
    // an offset between two atomics would also wait for the first atomic)
    int sv[kEnt], cv[kEnt];
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if ((rb + j * split) * 256 >= ne) break;
      const int t = (rb + j * split) * 256 + (int)threadIdx.x;
      const int pk = pkv[j];
      const int x = wrap1(ox + off_x(pk), G.nx), y = wrap1(oy + off_y(pk), G.ny), z = wrap1(oz + off_z(pk), G.nz);
      const int kind = entry_kind(pk);
      sv[j] = site_of(G, x, y, z);
      cv[j] = t < ne && kind != 3 && !wall_site(G, x, y, z) ? 2 * (e0 + t) + (kind == 2) : -1;
    }
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if ((rb + j * split) * 256 >= ne) break;
      if (cv[j] >= 0) atomicMin(&own[sv[j]], cv[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Near-contact closure (2D; not in the paper, which leaves lubrication
// untreated, section 2.3): one workgroup.  Pairs i < j of a box whose surface
// gap is below h_max at the start of the step are listed in lexicographic
// order (from the candidate lists), the network gives (a_n, a_t) for each
// pair on the matrix cores, 16 pairs per wave tile, and every particle sums
// mu U (a_n n + a_t t) over its pairs in list order (+ as i, - as j), with U
// = (u_i - u_j).n the approach speed.  The particle update adds it to the
// hydrodynamic force.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_closure(DevParticles P, int np, Boxes BX, const float* __restrict__ params,
                                                  double h_max, double mu, double tau, int* status) {
  __shared__ mlp::Weights w;
  __shared__ int s_i[kClosurePairs], s_j[kClosurePairs];
  __shared__ float s_a[kClosurePairs][2];
  __shared__ int s_scan[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  mlp::load_weights(w, params, tid, 256);
  __syncthreads();
  // list of close pairs
  int total = 0;
  for (int b = 0; b < np; b += 256) {
    const int p = b + tid;
    int c = 0;
    if (p < np) {
      const Geo G = geo_of(BX, P, p);
      for (int t = 0; t < P.cand_n[p]; t++) {
        const int j = P.cand[p * kCandMax + t];
        double dx = P.x[3 * j] - P.x[3 * p], dy = P.x[3 * j + 1] - P.x[3 * p + 1];
        dx -= G.nx * floor(dx / G.nx + 0.5);
        dy -= G.ny * floor(dy / G.ny + 0.5);
        c += sqrt(dx * dx + dy * dy) - P.rad[p] - P.rad[j] < h_max;
      }
    }
    int chunk;
    int at = total + block_excl_scan<256>(c, s_scan, chunk);
    if (c) {
      const Geo G = geo_of(BX, P, p);
      for (int t = 0; t < P.cand_n[p]; t++) {
        const int j = P.cand[p * kCandMax + t];
        double dx = P.x[3 * j] - P.x[3 * p], dy = P.x[3 * j + 1] - P.x[3 * p + 1];
        dx -= G.nx * floor(dx / G.nx + 0.5);
        dy -= G.ny * floor(dy / G.ny + 0.5);
        if (sqrt(dx * dx + dy * dy) - P.rad[p] - P.rad[j] < h_max) {
          if (at < kClosurePairs) {
            s_i[at] = p;
            s_j[at] = j;
          }
          at++;
        }
      }
    }
    total += chunk;
  }
  __syncthreads();  // the pair list is complete
  if (total > kClosurePairs) {
    if (tid == 0) atomicOr(status, kStatusClosure);
    total = kClosurePairs;
  }
  // the network on tiles of 16 pairs
  const int r = lane & 15, g = lane >> 4;
  for (int t0 = 16 * wv; t0 < total; t0 += 16 * 4) {
    const int t = t0 + r;
    mlp::h4 xb = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
    if (t < total && g < 2) {
      const int i = s_i[t], j = s_j[t];
      const Geo G = geo_of(BX, P, i);
      double dx = P.x[3 * j] - P.x[3 * i], dy = P.x[3 * j + 1] - P.x[3 * i + 1];
      dx -= G.nx * floor(dx / G.nx + 0.5);
      dy -= G.ny * floor(dy / G.ny + 0.5);
      float in[8];
      mlp::closure_inputs(P.x[3 * i], P.x[3 * i + 1], P.rad[i], P.rad[j], dx, dy, tau, in);
#pragma unroll
      for (int k = 0; k < 4; k++) xb[k] = (_Float16)in[4 * g + k];
    }
    mlp::h4 h1[4], h2[4];
    mlp::f4 y;
    mlp::forward_tile(w, xb, h1, h2, y, lane);
    if (g == 0 && t < total) {
      s_a[t][0] = y[0] + w.b3[0];
      s_a[t][1] = y[1] + w.b3[1];
    }
  }
  __syncthreads();
  // per-particle sums in list order
  for (int p = tid; p < np; p += 256) {
    double fx = 0, fy = 0;
    for (int t = 0; t < total; t++) {
      const int i = s_i[t], j = s_j[t];
      if (i != p && j != p) continue;
      const Geo G = geo_of(BX, P, i);
      double dx = P.x[3 * j] - P.x[3 * i], dy = P.x[3 * j + 1] - P.x[3 * i + 1];
      dx -= G.nx * floor(dx / G.nx + 0.5);
      dy -= G.ny * floor(dy / G.ny + 0.5);
      const double dist = sqrt(dx * dx + dy * dy);
      const double nx = dx / dist, ny = dy / dist;
      const double U = (P.u[3 * i] - P.u[3 * j]) * nx + (P.u[3 * i + 1] - P.u[3 * j + 1]) * ny;
      const double an = (double)s_a[t][0], at = (double)s_a[t][1];
      const double ffx = mu * U * (an * nx + at * -ny), ffy = mu * U * (an * ny + at * nx);
      if (i == p) {
        fx += ffx;
        fy += ffy;
      } else {
        fx -= ffx;
        fy -= ffy;
      }
    }
    P.fc[3 * p] = fx;
    P.fc[3 * p + 1] = fy;
    P.fc[3 * p + 2] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// K5: the IS substep of the step that just ran (pending = 1) and the ball-site
// records of the next sweep.
//  - IS substep at the new positions (eq. 12, fourth substep): every owned IS
//    site gets f^eq_i(rho_I, u_p' + omega_p' x r) for all i, written in place
//    into the post-collision state the next sweep pulls from.  rho_I is the
//    density this step's sweep kept at ball sites, or the sum of the site's
//    populations when its particle jumped along all three axes at once (the
//    site may then lie outside the ball the sweep kept densities for); the
//    owner reads them before it overwrites them, and no other thread touches
//    that site.
//  - Records: every entry at a ball site writes its flag, kSiteBS at an
//    owned BS site and kSiteBall elsewhere (the same value from every
//    writer, read off the owner map); the owning BS entry writes the site's
//    record: the rigid-body velocity of the next BS substep (eq. 5) and its
//    own index.
// ---------------------------------------------------------------------------
// Element of f*_i of site (x, y, z) of box G in a post-collision state of
// layout lay (kLayAB, or either half of the AA pattern).
template <int Q>
__device__ __forceinline__ size_t coll_index(int lay, int i, const Geo& G, int x, int y, int z) {
  using L = Lattice<Q>;
  if (lay == kLayAAStream)
    return (size_t)pop_elem(
        Q, i, site_of(G, wrap1(x + L::cx(i), G.nx), wrap1(y + L::cy(i), G.ny), wrap1(z + L::cz(i), G.nz)));
  return (size_t)pop_elem(Q, lay == kLayAASwap ? opposite<Q>(i) : i, site_of(G, x, y, z));
}

// Streaming store of one stored population value.
__device__ __forceinline__ void nt_put(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_put(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_put(_Float16* p, _Float16 v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_put(bf16s* p, bf16s v) { __builtin_nontemporal_store(v.v, (uint16_t*)p); }

// IS values of site s (offset o of particle p with the particle's velocities
// in the compute type; the value is stored in it).
template <int Q, typename T, bool NTS>
__device__ __forceinline__ void impose_is(T* __restrict__ S, int lay, const Geo& G, int x, int y, int z,
                                          double dr, typename Store<T>::C rx,
                                          typename Store<T>::C ry, typename Store<T>::C rz,
                                          typename Store<T>::C upx, typename Store<T>::C upy,
                                          typename Store<T>::C upz, typename Store<T>::C wx,
                                          typename Store<T>::C wy, typename Store<T>::C wz, double rho0) {
#pragma clang fp contract(off)
  using L = Lattice<Q>;
  using C = typename Store<T>::C;
  constexpr bool kRaw = std::is_same<T, _Float16>::value || std::is_same<T, bf16s>::value;
  const C inv_sig = (C)(1.0 / pop_unit<T>(1.0));
  const C vx = upx + (wy * rz - wz * ry);
  const C vy = upy + (wz * rx - wx * rz);
  const C vz = upz + (wx * ry - wy * rx);
  const C dc = (C)dr;
  const C rho = (C)rho0 + dc;
  const C usq = C(1.5) * fmac(vx, vx, fmac(vy, vy, vz * vz));
  [[maybe_unused]] const Feq16<Q, C> fe(dc, rho, usq, inv_sig);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    // f^eq_i - w_i rho0 as the sweep's BS substep writes it: for 16-bit
    // storage the stored number directly (the weight cancels), so the
    // encoding is one rounding of a compute-type value
    C e;
    if constexpr (kRaw) {
      e = fe(i, vx, vy, vz);
    } else {
      const C cu = dot_c<L>(i, vx, vy, vz);
      e = C(L::w(i)) * fmac(rho, fmac(C(4.5) * cu, cu, fmac(C(3), cu, -usq)), dc);
    }
    const T v = store_enc<T>(e);
    T* const dst = S + coll_index<Q>(lay, i, G, x, y, z);
    // NTS (the AA pattern, whose next sweep reads and rewrites these lines in
    // place): streaming stores keep the partly written lines out of the
    // caches; with two arrays they only move the same cost from the sweep here
    if constexpr (NTS)
      nt_put(dst, v);
    else
      *dst = v;
  }
}

// Record of site s owned by BS entry bs: rigid-body velocity u_q + omega_q x r
// and bs, into vel[4s..4s+3].
template <typename C>
__device__ __forceinline__ void store_bs_velocity(C* __restrict__ vel, int s, int bs, const DevParticles& P,
                                                  const DevEntries& E) {
  const int q = E.pid[bs];
  const int ok = E.off[bs];
  const double rx = (double)off_x(ok) - P.phi[3 * q], ry = (double)off_y(ok) - P.phi[3 * q + 1],
               rz = (double)off_z(ok) - P.phi[3 * q + 2];
  const double ax = P.om[3 * q], ay = P.om[3 * q + 1], az = P.om[3 * q + 2];
  vel[4 * (size_t)s] = (C)(P.u[3 * q] + (ay * rz - az * ry));
  vel[4 * (size_t)s + 1] = (C)(P.u[3 * q + 1] + (az * rx - ax * rz));
  vel[4 * (size_t)s + 2] = (C)(P.u[3 * q + 2] + (ax * ry - ay * rx));
  vel[4 * (size_t)s + 3] = idx_as<C>(bs);
}

template <int Q, typename T, bool NTS>
__global__ __launch_bounds__(256) void k_prepare(const int* __restrict__ own,
                                                  uint8_t* __restrict__ flag, typename Store<T>::C* __restrict__ vel,
                                                  double* __restrict__ slot,
                                                  const typename Store<T>::C* __restrict__ drho, T* __restrict__ S,
                                                  DevParticles P, DevEntries E, Boxes BX, int nent, double rho0,
                                                  int pending, int lay) {
  using C = typename Store<T>::C;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nent) return;
  const int p = E.pid[e];
  const Geo G = geo_of(BX, P, p);
  const int pk = E.off[e];
  int x, y, z;
  entry_xyz(P, G, p, pk, x, y, z);
  const int s = site_of(G, x, y, z);
  const int o = own[s];
  if (pending && o == 2 * e + 1) {
    double dr;
    if (P.jump[p]) {
      dr = 0;
#pragma unroll
      for (int j = 0; j < Q; j++) dr += (double)pop_ld<Q, T>(S + coll_index<Q>(lay, j, G, x, y, z), j);
    } else {
      dr = (double)drho[s];
    }
    impose_is<Q, T, NTS>(S, lay, G, x, y, z, dr, (C)((double)off_x(pk) - P.phi[3 * p]),
                    (C)((double)off_y(pk) - P.phi[3 * p + 1]),
                    (C)((double)off_z(pk) - P.phi[3 * p + 2]), (C)P.u[3 * p], (C)P.u[3 * p + 1], (C)P.u[3 * p + 2],
                    (C)P.om[3 * p], (C)P.om[3 * p + 1], (C)P.om[3 * p + 2], rho0);
  }
  // every entry at s writes the same flag, from the owner map
  flag[s] = o != kEmpty && !(o & 1) ? kSiteBS : kSiteBall;
  if (o == 2 * e) store_bs_velocity<C>(vel, s, e, P, E);  // the owner's record
  else if (entry_kind(pk) == 1) slot[4 * (size_t)e] = kSlotUnowned;
}

// ---------------------------------------------------------------------------
// K5 with kind grids (balls of at most kPrepareLocalMax bounding-box sites):
// the work of k_prepare, one to eight workgroups per particle (rows of
// kGridBlock entries dealt round-robin; entries in raster order, so the
// loads at their own sites are row-coalesced), with the owner of a site
// settled without an owner map.  A site is owned by the lowest particle id among those whose
// BS or IS entry lies on it at the new shifts (none on wall sites); only the
// particles listed as sharing candidates (k_reduce) can have such an entry on
// one of this particle's sites, and their kind grids say which.  Flags are
// written only where they can change: at the sites of a particle whose shift
// changed in this step (its new sites, and its old sites that no ball of it
// covers any more, cleared or handed to the neighbour covering them) and, with
// flags_all, at every ball site (after particles are added).  Every writer of
// a flag computes it from the same final map, so they agree.
// ---------------------------------------------------------------------------
// Kind of particle q's template at site (x, y, z) of its box, with q's
// origin (og) and kind-grid half-width R: 0 unless the site is one of its
// ball sites.  Template offsets are shorter than half the box, so the
// minimum-image offset is the only candidate.
template <int DIM>
__device__ __forceinline__ int kind_at(const uint8_t* __restrict__ kg, int R, int ox, int oy, int oz, const Geo& G,
                                       int x, int y, int z) {
  int dx = x - ox, dy = y - oy, dz = z - oz;
  dx += dx > G.nx / 2 ? -G.nx : (dx < -(G.nx / 2) ? G.nx : 0);
  dy += dy > G.ny / 2 ? -G.ny : (dy < -(G.ny / 2) ? G.ny : 0);
  dz += dz > G.nz / 2 ? -G.nz : (dz < -(G.nz / 2) ? G.nz : 0);
  if (dx < -R || dx > R || dy < -R || dy > R || dz < -R || dz > R) return 0;
  const int W = 2 * R + 1;
  return kg[DIM == 3 ? ((dz + R) * W + (dy + R)) * W + (dx + R) : (dy + R) * W + (dx + R)];
}

constexpr int kGridBlock = kPrepareBlock;

template <int Q, typename T, bool NTS>
__global__ __launch_bounds__(kGridBlock) void k_prepare_grid(uint8_t* __restrict__ flag,
                                                             typename Store<T>::C* __restrict__ vel,
                                                             double* __restrict__ slot,
                                                             const typename Store<T>::C* __restrict__ drho,
                                                             T* __restrict__ S, DevParticles P, DevEntries E, Boxes BX,
                                                             double rho0, int pending, int lay, int split,
                                                             int flags_all) {
  using C = typename Store<T>::C;
  constexpr int DIM = Q == 9 ? 2 : 3;
  __shared__ int s_nb[kNbrMax][6];  // neighbour id, origin, kind-grid start and half-width
  const int p = blockIdx.x / split, part = blockIdx.x % split;
  const int tid = threadIdx.x;
  const Geo G = geo_of(BX, P, p);
  const int ox0 = P.org[3 * p], oy0 = P.org[3 * p + 1], oz0 = P.org[3 * p + 2];
  const double phx = P.phi[3 * p], phy = P.phi[3 * p + 1], phz = P.phi[3 * p + 2];
  const double upx = P.u[3 * p], upy = P.u[3 * p + 1], upz = P.u[3 * p + 2];
  const double wx = P.om[3 * p], wy = P.om[3 * p + 1], wz = P.om[3 * p + 2];
  const C cupx = (C)upx, cupy = (C)upy, cupz = (C)upz, cwx = (C)wx, cwy = (C)wy, cwz = (C)wz;
  const bool jump = P.jump[p] != 0;
  const bool moved = P.moved[p] != 0;
  const bool flags = flags_all != 0 || moved;
  // interior entries come last and only write flags: skipped when the flags
  // stand as they are
  const int e0 = P.ent0[p], ne = P.nbs[p] + P.nis[p] + (flags ? P.nin[p] : 0);
  const int nn = P.nbr_n[p];
  const int Rp = P.kgR[p];
  const uint8_t* kgp = P.kgrid + P.kg0[p];
  if (nn > 0) {
    for (int t = tid; t < nn; t += kGridBlock) {
      const int q = P.nbr[(size_t)p * kNbrMax + t];
      s_nb[t][0] = q;
      s_nb[t][1] = P.org[3 * q];
      s_nb[t][2] = P.org[3 * q + 1];
      s_nb[t][3] = P.org[3 * q + 2];
      s_nb[t][4] = P.kg0[q];
      s_nb[t][5] = P.kgR[q];
    }
    __syncthreads();
  }
  // owner (lowest id claiming the site, INT_MAX for none) and its kind at
  // (x, y, z), given this particle's own kind there (0 if none); cov: some
  // ball covers the site
  auto settle = [&](int x, int y, int z, int kp, int& oid, int& okind, bool& cov) {
    const bool wall = G.walls && wall_site(G, x, y, z);
    oid = INT_MAX;
    okind = 0;
    cov = kp != 0;
    if (!wall && (kp == 1 || kp == 2)) {
      oid = p;
      okind = kp;
    }
    for (int t = 0; t < nn; t++) {
      const int q = s_nb[t][0];
      if (q > oid && cov) break;  // ascending ids: no lower claimer left
      const int kq = kind_at<DIM>(P.kgrid + s_nb[t][4], s_nb[t][5], s_nb[t][1], s_nb[t][2], s_nb[t][3], G, x, y, z);
      cov = cov || kq != 0;
      if (!wall && (kq == 1 || kq == 2) && q < oid) {
        oid = q;
        okind = kq;
      }
    }
  };
  // The entries come kind by kind (BS, IS, interior), so they are dealt in
  // runs of 64 (one wave each) round-robin over the particle's split
  // workgroups, which then share the IS substep's stores evenly: run c goes
  // to workgroup c % split, whose waves take its runs in turn.
  constexpr int kEnt = 4;
  const int wv = tid >> 6, lane = tid & 63;
  constexpr int kWv = kGridBlock / 64;
  auto run0 = [&](int m) { return (part + split * (kWv * m + wv)) * 64; };  // this wave's m-th run
  for (int mb = 0; (part + split * kWv * mb) * 64 < ne; mb += kEnt) {
    int pkv[kEnt];
    C dv[kEnt];
    int sv[kEnt];
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if (run0(mb + j) >= ne) break;  // the same for the whole wave
      pkv[j] = E.off[e0 + min(run0(mb + j) + lane, ne - 1)];
    }
#pragma unroll
    for (int j = 0; j < kEnt; j++) {
      if (run0(mb + j) >= ne) break;
      const int pk = pkv[j];
      sv[j] = site_of(G, wrap1(ox0 + off_x(pk), G.nx), wrap1(oy0 + off_y(pk), G.ny), wrap1(oz0 + off_z(pk), G.nz));
      // used only at an IS site the substep claims: runs of BS entries (the
      // first of a particle's entries) load nothing
      dv[j] = entry_kind(pk) == 2 ? drho[sv[j]] : C(0);
    }
#pragma unroll 1
    for (int j = 0; j < kEnt; j++) {
      const int t = run0(mb + j) + lane;
      if (t >= ne) continue;
      const int e = e0 + t;
      const int pk = pkv[j];
      const int ox = off_x(pk), oy = off_y(pk), oz = off_z(pk), kp = entry_kind(pk);
      const int s = sv[j];
      const int sxx = wrap1(ox0 + ox, G.nx), syy = wrap1(oy0 + oy, G.ny), szz = wrap1(oz0 + oz, G.nz);
      int oid, okind;
      bool cov;
      settle(sxx, syy, szz, kp, oid, okind, cov);
      const bool mine = oid == p;
      if (pending && mine && kp == 2) {
        double dr;
        if (jump) {
          dr = 0;
#pragma unroll
          for (int k = 0; k < Q; k++) dr += (double)pop_ld<Q, T>(S + coll_index<Q>(lay, k, G, sxx, syy, szz), k);
        } else {
          dr = (double)dv[j];
        }
        impose_is<Q, T, NTS>(S, lay, G, sxx, syy, szz, dr, (C)((double)ox - phx), (C)((double)oy - phy),
                             (C)((double)oz - phz), cupx, cupy, cupz, cwx, cwy, cwz, rho0);
      }
      if (flags) flag[s] = okind == 1 ? kSiteBS : kSiteBall;
      if (mine && kp == 1) {
        const double rx = (double)ox - phx, ry = (double)oy - phy, rz = (double)oz - phz;
        vel[4 * (size_t)s] = (C)(upx + (wy * rz - wz * ry));
        vel[4 * (size_t)s + 1] = (C)(upy + (wz * rx - wx * rz));
        vel[4 * (size_t)s + 2] = (C)(upz + (wx * ry - wy * rx));
        vel[4 * (size_t)s + 3] = idx_as<C>(e);
      } else if (kp == 1) {
        slot[4 * (size_t)e] = kSlotUnowned;  // a BS entry whose site another particle or a wall holds
      }
      if (moved) {
        // the site this entry held before the translation: cleared unless a
        // ball still covers it (this particle's new ball covers it through
        // one of its own entries, which writes the flag there)
        const int xo = wrap1(P.orgp[3 * p] + ox, G.nx), yo = wrap1(P.orgp[3 * p + 1] + oy, G.ny),
                  zo = wrap1(P.orgp[3 * p + 2] + oz, G.nz);
        if (kind_at<DIM>(kgp, Rp, ox0, oy0, oz0, G, xo, yo, zo) == 0) {
          int qo, qk;
          bool qc;
          settle(xo, yo, zo, 0, qo, qk, qc);
          flag[site_of(G, xo, yo, zo)] = !qc ? 0 : (qk == 1 ? kSiteBS : kSiteBall);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Read-out and set-up kernels (off the step loop).
// ---------------------------------------------------------------------------
// Moments of sites s0 .. s0 + cnt - 1 of box G (box-local indices).
template <int Q, typename T>
__global__ void k_moments(const T* __restrict__ A, double* __restrict__ rho, double* __restrict__ u,
                          Geo G, double rho0, int64_t s0, int64_t cnt, int lay) {
  using L = Lattice<Q>;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= cnt) return;
  const int64_t s = s0 + idx;
  const int x = (int)(s % G.nx), y = (int)((s / G.nx) % G.ny), z = (int)(s / ((int64_t)G.nx * G.ny));
  double drho = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; i++) {
    // f_i arriving at x (the three state layouts)
    const bool here = lay == kLayAAStream;
    const int sx = here ? x : wrap(x - L::cx(i), G.nx), sy = here ? y : wrap(y - L::cy(i), G.ny),
              sz = here ? z : wrap(z - L::cz(i), G.nz);
    const int plane = lay == kLayAASwap ? opposite<Q>(i) : i;
    const double g = (double)pop_ld<Q, T>(A + pop_elem(Q, plane, site_of(G, sx, sy, sz)), i);
    drho += g;
    j[0] += L::cx(i) * g;
    j[1] += L::cy(i) * g;
    j[2] += L::cz(i) * g;
  }
  const double r = rho0 + drho;
  rho[idx] = r;
  for (int a = 0; a < 3; a++) u[3 * idx + a] = j[a] / r;
}

// B_i(s) = A_i(s - dir * c_i) over the sites of box G: dir = +1 pulls
// (state -> post-stream f), dir = -1 pushes (post-stream f -> state).
template <int Q, typename T>
__global__ void k_shift(const T* __restrict__ A, T* __restrict__ B, Geo G, int dir) {
  using L = Lattice<Q>;
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= G.N) return;
  const int x = (int)(s % G.nx), y = (int)((s / G.nx) % G.ny), z = (int)(s / ((int64_t)G.nx * G.ny));
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int sx = wrap(x - dir * L::cx(i), G.nx), sy = wrap(y - dir * L::cy(i), G.ny),
              sz = wrap(z - dir * L::cz(i), G.nz);
    B[pop_elem(Q, i, G.off + s)] = A[pop_elem(Q, i, site_of(G, sx, sy, sz))];
  }
}

template <typename V>
__global__ void k_fill(V* __restrict__ p, int64_t n, V v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Every site record at rest and naming no entry (index -1), so that a record
// the prepare pass never wrote can never be taken for a valid one.
template <typename C>
__global__ void k_fill_records(C* __restrict__ vel, int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  vel[4 * s] = C(0);
  vel[4 * s + 1] = C(0);
  vel[4 * s + 2] = C(0);
  vel[4 * s + 3] = idx_as<C>(-1);
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// one 16-byte vector per thread, streaming store; NTL: streaming load too
// (the access kinds of the one-box sweeps, fastest from HBM), else a plain
// load (the ensemble sweep's, fastest from the last-level cache)
template <bool NTL>
__global__ __launch_bounds__(256) void k_copy16(const v4u* __restrict__ src, v4u* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(NTL ? __builtin_nontemporal_load(src + i) : src[i], dst + i);
}

inline unsigned blocks_for(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
struct Layout {
  size_t f[2], drho, own, flag, status, stage;
  size_t x, x0, u, om, phi, fext, dP, dL, F, T, m, I, rad, b0, k, org, ent0, nbs, nis, nin, jump, box, cand_n, cand,
      pairs;
  size_t orgp, moved, kg0, kgR, nbr_n, nbr, kgrid;
  size_t off, pid, slot, vel;
  size_t boxes, fbt, tiles, fc, clo;
  int64_t max_ent, max_tiles;
  size_t total;
};

// The boxes of a context: one for lbm_create, several for an ensemble.
struct BoxSet {
  std::vector<int> dims;  // [nbox][3]
  int64_t NT = 0;         // all sites
  int64_t max_tiles = 0;  // tiles of the narrowest tile width
};

constexpr int kTileMin = 64;

BoxSet make_boxset(int nbox, const int32_t* dims) {
  BoxSet b;
  b.dims.assign(dims, dims + 3 * (size_t)nbox);
  for (int i = 0; i < nbox; i++) {
    const int64_t nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
    b.NT += nx * ny * nz;
    b.max_tiles += (nx * ny * nz + kTileMin - 1) / kTileMin + 1;  // + the short first tile
  }
  return b;
}

size_t store_size(int storage) { return storage == LBM_FP64 ? 8 : storage == LBM_FP32 ? 4 : 2; }

// Sites of the population array: the sites rounded up to whole blocks (see
// pop_elem); the array holds q times as many values.
int64_t pop_stride(int64_t sites) { return (sites + kPopBlock - 1) / kPopBlock * kPopBlock; }

// One population of the array spans at most 4 GiB (N sizeof(T) <= 2^32): a
// limit of the interface, which caps FP64 boxes at 2^29 sites and 16-bit
// ones at the 2^31 sites the 32-bit site indices of the kernels allow.
bool plane_fits(int storage, int64_t sites) { return (uint64_t)sites * store_size(storage) <= ((uint64_t)1 << 32); }

// Bytes of one particle's kind grid: offsets of a template lie within
// floor(r + 1/2) of its origin along every axis (|o - phi| <= r, |phi| <= 1/2).
int kind_grid_half(double r) { return (int)std::floor(r + 0.5); }
size_t kind_grid_bytes(int dim, double r) {
  const size_t w = 2 * (size_t)kind_grid_half(r) + 1;
  return dim == 2 ? w * w : w * w * w;
}

// Balls whose bounding box holds at most kPrepareLocalMax sites take the
// per-particle kernels and settle site ownership from kind grids; larger ones
// keep an owner map that every step rebuilds, and a prepare pass with one
// thread per entry.
bool uses_kind_grids(int dim, double rmax) { return kind_grid_bytes(dim, rmax) <= (size_t)kPrepareLocalMax; }

int64_t entries_per_particle(int dim, double rmax) {
  const int64_t e = 2 * (int64_t)std::ceil(rmax) + 1;
  return dim == 2 ? e * e : e * e * e;
}

Layout make_layout(const lbm_params& p, const BoxSet& bs) {
  Layout L{};
  const int64_t N = bs.NT;
  const int64_t nbox = (int64_t)bs.dims.size() / 3;
  const int dim = p.lattice == LBM_D2Q9 ? 2 : 3;
  const int64_t np = std::max<int64_t>(p.max_particles, 1);
  L.max_ent = np * entries_per_particle(dim, p.max_radius);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t at = cur;
    cur += (bytes + kAlign - 1) / kAlign * kAlign;
    return at;
  };
  const size_t fb = (size_t)p.lattice * pop_stride(N) * store_size(p.storage);
  L.f[0] = take(fb);
  L.f[1] = p.aa ? L.f[0] : take(fb);  // the AA pattern updates one array in place
  L.drho = take((size_t)N * (p.storage == LBM_FP64 ? 8 : 4));
  L.own = take(sizeof(int) * N);
  L.flag = take(N);
  L.status = take(64);
  // moments staging of field read-outs (two arrays stage in the idle one)
  L.stage = p.aa ? take(4 * sizeof(double) * (size_t)std::min<int64_t>(N, (int64_t)1 << 20)) : 0;
  const size_t v3 = sizeof(double) * 3 * np, v1 = sizeof(double) * np;
  L.x = take(v3); L.x0 = take(v3); L.u = take(v3); L.om = take(v3); L.phi = take(v3);
  L.fext = take(v3); L.dP = take(v3); L.dL = take(v3); L.F = take(v3); L.T = take(v3);
  L.m = take(v1); L.I = take(v1); L.rad = take(v1);
  L.b0 = take(sizeof(int) * 3 * np); L.k = take(sizeof(int) * 3 * np); L.org = take(sizeof(int) * 3 * np);
  L.ent0 = take(sizeof(int) * np); L.nbs = take(sizeof(int) * np); L.nis = take(sizeof(int) * np);
  L.nin = take(sizeof(int) * np);
  L.jump = take(sizeof(int) * np);
  L.orgp = take(sizeof(int) * 3 * np);
  L.moved = take(sizeof(int) * np);
  L.kg0 = take(sizeof(int) * np);
  L.kgR = take(sizeof(int) * np);
  L.nbr_n = take(sizeof(int) * np);
  L.nbr = take(sizeof(int) * np * kNbrMax);
  L.kgrid = take(uses_kind_grids(dim, p.max_radius) ? (size_t)np * kind_grid_bytes(dim, p.max_radius) : 0);
  L.box = take(sizeof(int) * np);
  L.cand_n = take(sizeof(int) * np);
  L.cand = take(sizeof(int) * np * kCandMax);
  L.pairs = take(sizeof(int) * 2 * np * kCandMax);
  L.off = take(sizeof(int) * L.max_ent);
  L.pid = take(sizeof(int) * L.max_ent);
  L.slot = take(sizeof(double) * 4 * L.max_ent);
  L.vel = take((p.storage == LBM_FP64 ? 8 : 4) * 4 * N);
  L.boxes = take(sizeof(Geo) * nbox);
  L.fbt = take(sizeof(double) * p.lattice * nbox);
  L.max_tiles = bs.max_tiles;
  L.tiles = take(3 * sizeof(int4) * bs.max_tiles);
  L.fc = take(sizeof(double) * 3 * np);
  L.clo = take(sizeof(float) * mlp::kParams);
  L.total = cur;
  return L;
}

int check_params(const lbm_params* p);

// Parameters of an ensemble: those of every box (prm with the box's size).
int check_boxes(const lbm_params* p, int nbox, const int32_t* dims) {
  if (!p || nbox < 1 || !dims) return LBM_EINVAL;
  int64_t NT = 0;
  for (int b = 0; b < nbox; b++) {
    lbm_params q = *p;
    q.nx = dims[3 * b];
    q.ny = dims[3 * b + 1];
    q.nz = dims[3 * b + 2];
    const int rc = check_params(&q);
    if (rc != LBM_OK) return rc;
    NT += (int64_t)q.nx * q.ny * q.nz;
  }
  if (NT >= ((int64_t)1 << 31) || !plane_fits(p->storage, NT)) return LBM_EINVAL;
  return LBM_OK;
}

int check_params(const lbm_params* p) {
  if (!p) return LBM_EINVAL;
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return LBM_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBM_EINVAL;
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return LBM_EINVAL;
  if ((int64_t)p->nx * p->ny * p->nz >= ((int64_t)1 << 31)) return LBM_EINVAL;
  if (p->storage >= LBM_FP64 && p->storage <= LBM_BF16 && !plane_fits(p->storage, (int64_t)p->nx * p->ny * p->nz))
    return LBM_EINVAL;
  if (!std::isfinite(p->tau) || !std::isfinite(p->rho0) || !std::isfinite(p->max_radius)) return LBM_ENONFINITE;
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(p->gravity[a]) || !std::isfinite(p->body_force[a])) return LBM_ENONFINITE;
  if (!(p->tau > 0.5) || !(p->rho0 > 0)) return LBM_EINVAL;
  if (p->max_particles < 0) return LBM_EINVAL;
  if (!(p->max_radius > 0) || p->max_radius > 120) return LBM_EINVAL;
  const int dim = p->lattice == LBM_D2Q9 ? 2 : 3;
  if (std::max<int64_t>(p->max_particles, 1) * entries_per_particle(dim, p->max_radius) > kMaxEntries)
    return LBM_ECAPACITY;
  if (p->storage < LBM_FP64 || p->storage > LBM_BF16) return LBM_EINVAL;
  if (p->walls < 0 || p->walls >= (1 << dim)) return LBM_EINVAL;
  if (p->aa != 0 && p->aa != 1) return LBM_EINVAL;
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < dim; a++) {
    if (!((p->walls >> a) & 1)) continue;
    if (n[a] < 5) return LBM_EINVAL;
    for (int hi = 0; hi < 2; hi++) {
      for (int k = 0; k < 3; k++)
        if (!std::isfinite(p->wall_velocity[a][hi][k])) return LBM_ENONFINITE;
      if (p->wall_velocity[a][hi][a] != 0.0) return LBM_EINVAL;  // walls slide tangentially
    }
  }
  return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct lbm_ctx {
  lbm_params prm;
  int q, dim;
  Geo G;                    // box 0 (the box of a single-box context)
  int nbox;
  int64_t NT;               // sites of all boxes
  int64_t PS;               // sites of the population array (see pop_stride)
  std::vector<Geo> boxes;   // host copy of the box table
  Geo* d_boxes;
  void* d_fbt;              // [nbox][q] 3 w_i c_i . f_b per box, compute type
  int4* d_tiles;
  int64_t ntiles;           // tiles of the current tile width
  int tiles_w;              // tile width the table was built for (0: none)
  int sweep_w, sweep_grid;  // sweep launch shape: w = 0 the one-box kernel, else tile width; grid 0 = one per tile
  int sweep_occ;            // cap on resident sweep workgroups per CU (0: none)
  int lds_cu, lds_block;    // LDS bytes per CU and the most one workgroup may reserve
  int device;               // the device the context was created on
  bool row_ok;              // one box whose rows fit the row kernel's (x-blocks, y, z) grid
  std::vector<int> h_box;   // box of every particle
  std::vector<double> fbb;  // [nbox][3] fluid body force density
  // step graph
  hipStream_t cap;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  int g_steps, g_cur, g_w, g_grid, g_occ;
  int64_t g_np, g_nent;
  int graph_steps;          // 0: eager launches
  int closure;              // near-contact closure network on
  double clo_h;             // gap below which it acts
  float* d_clo;             // its parameters
  hipStream_t stream;
  char* ws;
  Layout L;
  void* f[2];
  int cur;  // f[cur] holds the post-collision state of the last step
  void* drho;
  double* slot;
  void* vel;
  int* own;   // owner map: lowest BS/IS entry per site
  uint8_t* flag;  // [site]: 0, kSiteBall or kSiteBS
  int* status;
  DevParticles P;
  DevEntries E;
  int np;
  int64_t nent;
  std::vector<double> h_x0, h_rad, h_m, h_I, h_fext;
  std::vector<int> h_off, h_pid, h_nbs, h_nis, h_nin;
  bool grids;         // kind grids settle ownership in the per-particle prepare (else an
                      // owner map rebuilt every step and one thread per entry)
  size_t kg_used;     // bytes of kind grids in use
  int prep_split;     // most workgroups per particle of the per-particle prepare
  bool small_ball;    // the largest ball holds at most kSmallBall entries
  bool prof;
  bool failed;  // a HIP error left the device state part-way through an update
  std::vector<hipEvent_t> ev;
  size_t ev_used;
};

// Layout of the state between steps: the AA pattern alternates its two
// halves with the step parity (cur), kept like the buffer index of two arrays.
int state_layout(const lbm_ctx* c) { return c->prm.aa ? (c->cur == 0 ? kLayAAStream : kLayAASwap) : kLayAB; }

// Launch shapes: widths 64..512 are the tile kernel, 0 the row kernel of one box.
bool tile_width(int w) { return w == 64 || w == 128 || w == 256 || w == 512; }

#define HIP_TRY(expr)                          \
  do {                                         \
    if ((expr) != hipSuccess) return LBM_EHIP; \
  } while (0)

namespace {

template <int Q, typename T>
SiteArgs<T> site_args(lbm_ctx* c) {
  SiteArgs<T> sa;
  sa.flag = c->flag;
  sa.vel = (const typename Store<T>::C*)c->vel;
  sa.slot = c->slot;
  sa.drho = (typename Store<T>::C*)c->drho;
  sa.nent = (int)c->nent;
  sa.status = c->status;
  return sa;
}

Boxes boxes_arg(const lbm_ctx* c) {
  Boxes b;
  b.g0 = c->boxes[0];
  b.tab = c->d_boxes;
  b.nbox = c->nbox;
  return b;
}

// The IS substep of the step that just ran (pending = 1) and the records of
// every ball site for the next sweep.  Up to eight workgroups per particle for
// balls of moderate size, one thread per entry otherwise.
template <int Q, typename T, bool NTS>
int launch_prepare_as(lbm_ctx* c, int pending, int flags_all) {
  using C = typename Store<T>::C;
  if (c->grids) {
    // split workgroups per particle only while the particles alone leave the
    // GPU short of workgroups (about 8 per CU)
    const int split = std::max(1, std::min(c->prep_split, 2048 / std::max(c->np, 1)));
    k_prepare_grid<Q, T, NTS><<<c->np * split, kGridBlock, 0, c->stream>>>(
        c->flag, (C*)c->vel, c->slot, (const C*)c->drho, (T*)c->f[c->cur], c->P, c->E, boxes_arg(c), c->prm.rho0,
        pending, state_layout(c), split, flags_all);
  } else {
    k_prepare<Q, T, NTS><<<blocks_for(c->nent), 256, 0, c->stream>>>(
        c->own, c->flag, (C*)c->vel, c->slot, (const C*)c->drho, (T*)c->f[c->cur], c->P, c->E, boxes_arg(c),
        (int)c->nent, c->prm.rho0, pending, state_layout(c));
  }
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <int Q, typename T>
int launch_prepare(lbm_ctx* c, int pending, int flags_all) {
  if (c->nent == 0) return LBM_OK;
  // Streaming IS stores for the AA pattern (the in-place sweep pays most for
  // partly written lines) and for two arrays small enough to stay in the
  // last-level cache (D2Q9 1024^2, 75 MB: step 33.2 -> 32.0 us); larger
  // two-array states keep plain stores (256^3 FP32: 0.456 against 0.464 ms).
  const size_t both = 2 * (size_t)c->q * c->PS * store_size(c->prm.storage);
  const bool nts = state_layout(c) != kLayAB || both <= kCacheResidentBytes;
  return nts ? launch_prepare_as<Q, T, true>(c, pending, flags_all)
             : launch_prepare_as<Q, T, false>(c, pending, flags_all);
}

// Tile list {box, y, z, x0} of width w, box by box, rows in z, y order.
// FP64 bits of v as {lo, hi} ints.
static void dbl_bits(double v, int& lo, int& hi) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  lo = (int)(uint32_t)(u & 0xffffffffu);
  hi = (int)(uint32_t)(u >> 32);
}

int build_tiles(lbm_ctx* c, int w) {
  if (c->tiles_w == w) return LBM_OK;
  std::vector<int4> t;
  for (int b = 0; b < c->nbox; b++) {
    const Geo& g = c->boxes[b];
    int4 inv;
    dbl_bits(1.0 / g.nx, inv.x, inv.y);
    dbl_bits(1.0 / g.ny, inv.z, inv.w);
    // tiles start at multiples of w of the whole site range, so that the
    // streaming stores of a tile fill whole cache lines (boxes start
    // anywhere); a box's first tile runs up to the first such multiple
    const int64_t head = (w - g.off % w) % w;
    for (int64_t s0 = 0; s0 < g.N;) {
      const int64_t s1 = std::min<int64_t>(g.N, s0 == 0 && head > 0 ? head : s0 + w);
      t.push_back(make_int4(b, (int)s0, (int)s1, 0));
      t.push_back(make_int4(g.nx, g.ny, g.nz, (int)g.off));
      t.push_back(inv);
      s0 = s1;
    }
  }
  if ((int64_t)t.size() > 3 * c->L.max_tiles) return LBM_EINVAL;
  HIP_TRY(hipMemcpyAsync(c->d_tiles, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->ntiles = (int64_t)t.size() / 3;
  c->tiles_w = w;
  return LBM_OK;
}

template <int Q, typename T>
SweepArgs<Q, typename Store<T>::C> sweep_args(const lbm_ctx* c) {
  using C = typename Store<T>::C;
  using Lt = Lattice<Q>;
  SweepArgs<Q, C> a;
  a.nx = c->G.nx;
  a.ny = c->G.ny;
  a.nz = c->G.nz;
  a.nxb = (c->G.nx + kSweepBlock - 1) / kSweepBlock;
  a.omega = (C)(1.0 / c->prm.tau);
  a.rho0 = (C)c->prm.rho0;
  a.walls = c->prm.walls;
  for (int ax = 0; ax < 3; ax++)
    for (int hi = 0; hi < 2; hi++)
      for (int k = 0; k < 3; k++) a.wu[ax][hi][k] = (C)((c->prm.walls >> ax) & 1 ? c->prm.wall_velocity[ax][hi][k] : 0.0);
  for (int i = 0; i < Q; i++) {
    const double cf = Lt::cx(i) * c->fbb[0] + Lt::cy(i) * c->fbb[1] + Lt::cz(i) * c->fbb[2];
    a.fbt[i] = (C)(3.0 * Lt::w(i) * cf);
  }
  return a;
}

// One sweep in the context's launch shape.
// LDS each sweep workgroup reserves so that at most occ of them are resident
// on one CU (0 for no cap), in whole KiB; occ_ok: the amount fits one
// workgroup's limit.
size_t sweep_lds(const lbm_ctx* c, int occ) { return occ > 0 ? (size_t)(c->lds_cu / occ) & ~(size_t)1023 : 0; }
bool occ_ok(const lbm_ctx* c, int occ) {
  return occ == 0 || (occ > 0 && occ <= 32 && sweep_lds(c, occ) >= 1024 && sweep_lds(c, occ) <= (size_t)c->lds_block);
}

template <int Q, typename T, int LAY>
int launch_sweep_as(lbm_ctx* c, int w, int grid, int occ) {
  using C = typename Store<T>::C;
  // the occupancy cap: LDS reserved (not used) by every workgroup
  const size_t lds = sweep_lds(c, occ);
  const SweepArgs<Q, C> a = sweep_args<Q, T>(c);
  const T* A = (const T*)c->f[c->cur];
  T* B = (T*)c->f[1 - c->cur];  // the same array under the AA pattern
  const SiteArgs<T> sa = site_args<Q, T>(c);
  if (w == 0) {
    if constexpr (sizeof(T) == 2 && LAY == kLayAB) {
      if (a.nx % 2 == 0) {  // two sites per lane: one wave per 128 sites of a row
        const int64_t waves = (int64_t)((a.nx + kPairRow - 1) / kPairRow) * c->G.ny * c->G.nz;
        const unsigned g = (unsigned)((waves + kSweepBlock / 64 - 1) / (kSweepBlock / 64));
        if (c->np > 0)
          k_sweep_pairs<Q, T, true><<<g, kSweepBlock, lds, c->stream>>>(A, B, a, sa);
        else
          k_sweep_pairs<Q, T, false><<<g, kSweepBlock, lds, c->stream>>>(A, B, a, sa);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
      }
    }
    const dim3 grid3((unsigned)a.nxb, (unsigned)c->G.ny, (unsigned)c->G.nz);
    if (c->np > 0)
      k_sweep<Q, T, true, LAY><<<grid3, kSweepBlock, lds, c->stream>>>(A, B, a, sa);
    else
      k_sweep<Q, T, false, LAY><<<grid3, kSweepBlock, lds, c->stream>>>(A, B, a, sa);
  } else {
    const int64_t nt = c->ntiles;
    const unsigned g = (unsigned)(grid > 0 && grid < nt ? grid : nt);
    // streaming loads for one box, cached ones for an ensemble
    const bool one = c->nbox == 1;
    if (c->np > 0 && one)
      k_sweep_tiles<Q, T, true, LAY, true><<<g, w, lds, c->stream>>>(A, B, a, sa, c->d_tiles, (int)nt,
                                                                      (const C*)c->d_fbt);
    else if (c->np > 0)
      k_sweep_tiles<Q, T, true, LAY, false><<<g, w, lds, c->stream>>>(A, B, a, sa, c->d_tiles, (int)nt,
                                                                       (const C*)c->d_fbt);
    else if (one)
      k_sweep_tiles<Q, T, false, LAY, true><<<g, w, lds, c->stream>>>(A, B, a, sa, c->d_tiles, (int)nt,
                                                                       (const C*)c->d_fbt);
    else
      k_sweep_tiles<Q, T, false, LAY, false><<<g, w, lds, c->stream>>>(A, B, a, sa, c->d_tiles, (int)nt,
                                                                        (const C*)c->d_fbt);
  }
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}
template <int Q, typename T>
int launch_sweep(lbm_ctx* c, int w, int grid, int occ) {
  switch (state_layout(c)) {
    case kLayAAStream: return launch_sweep_as<Q, T, kLayAAStream>(c, w, grid, occ);
    case kLayAASwap: return launch_sweep_as<Q, T, kLayAASwap>(c, w, grid, occ);
    default: return launch_sweep_as<Q, T, kLayAB>(c, w, grid, occ);
  }
}

template <int Q, typename T>
int launch_step(lbm_ctx* c) {
  if (c->prof) {
    if (c->ev_used + 2 > c->ev.size()) {
      for (int t = 0; t < 64; t++) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->ev.push_back(e);
      }
    }
    HIP_TRY(hipEventRecord(c->ev[c->ev_used], c->stream));
  }
  const int rc = launch_sweep<Q, T>(c, c->sweep_w, c->sweep_grid, c->sweep_occ);
  if (rc != LBM_OK) return rc;
  if (c->prof) {
    HIP_TRY(hipEventRecord(c->ev[c->ev_used + 1], c->stream));
    c->ev_used += 2;
  }
  if (c->np > 0) {
    const Boxes bx = boxes_arg(c);
    const double margin = c->closure ? std::max(kMargin, c->clo_h) : kMargin;
    // half-size workgroups for many small balls: two waves then hold every
    // entry, and twice as many particles' workgroups fit the GPU at once
    if (c->small_ball && c->np > 1024) {
      if (c->grids)
        k_reduce<128, true><<<c->np, 128, 0, c->stream>>>(c->own, c->flag, c->slot, c->P, c->E, bx, c->prm.rho0,
                                                          margin, c->status);
      else
        k_reduce<128, false><<<c->np, 128, 0, c->stream>>>(c->own, c->flag, c->slot, c->P, c->E, bx, c->prm.rho0,
                                                           margin, c->status);
    } else {
      if (c->grids)
        k_reduce<kBoundaryBlock, true><<<c->np, kBoundaryBlock, 0, c->stream>>>(c->own, c->flag, c->slot, c->P, c->E,
                                                                                bx, c->prm.rho0, margin, c->status);
      else
        k_reduce<kBoundaryBlock, false><<<c->np, kBoundaryBlock, 0, c->stream>>>(
            c->own, c->flag, c->slot, c->P, c->E, bx, c->prm.rho0, margin, c->status);
    }
    if (c->closure)
      k_closure<<<1, 256, 0, c->stream>>>(c->P, c->np, bx, c->d_clo, c->clo_h,
                                          c->prm.rho0 * (c->prm.tau - 0.5) / 3.0, c->prm.tau, c->status);
    if (c->nbox == 1)
      k_particles<kParticleBlock><<<1, kParticleBlock, 0, c->stream>>>(c->P, c->dim, bx, c->status);
    else
      k_particles<kBoxParticleBlock><<<c->nbox, kBoxParticleBlock, 0, c->stream>>>(c->P, c->dim, bx, c->status);
    if (!c->grids) {
      const int split = std::max(1, std::min(c->prep_split, 2048 / std::max(c->np, 1)));  // as for prepare
      k_stamp_particles<<<c->np * split, 256, 0, c->stream>>>(c->own, c->P, c->E, bx, split);
    }
    HIP_TRY(hipGetLastError());
  }
  c->cur = 1 - c->cur;  // f[cur] now holds this step's post-collision state
  if (c->np > 0) return launch_prepare<Q, T>(c, 1, 0);
  return LBM_OK;
}

template <int Q, typename T>
int launch_moments(lbm_ctx* c, int box, double* d_rho, double* d_u, int64_t s0, int64_t cnt) {
  k_moments<Q, T><<<blocks_for(cnt), 256, 0, c->stream>>>((const T*)c->f[c->cur], d_rho, d_u, c->boxes[box],
                                                          c->prm.rho0, s0, cnt, state_layout(c));
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <int Q, typename T>
int launch_shift(lbm_ctx* c, const void* A, void* B, int dir) {
  for (int b = 0; b < c->nbox; b++)
    k_shift<Q, T><<<blocks_for(c->boxes[b].N), 256, 0, c->stream>>>((const T*)A, (T*)B, c->boxes[b], dir);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

#define DISPATCH_Q(c, Qv, FN, ...)                                                        \
  ((c)->prm.storage == LBM_FP64   ? FN<Qv, double>(__VA_ARGS__)                             \
   : (c)->prm.storage == LBM_FP32 ? FN<Qv, float>(__VA_ARGS__)                              \
   : (c)->prm.storage == LBM_FP16 ? FN<Qv, _Float16>(__VA_ARGS__)                           \
                                  : FN<Qv, bf16s>(__VA_ARGS__))
#define DISPATCH(c, FN, ...) ((c)->q == 9 ? DISPATCH_Q(c, 9, FN, __VA_ARGS__) : DISPATCH_Q(c, 19, FN, __VA_ARGS__))

double lattice_w(int q, int i) { return q == 9 ? Lattice<9>::w(i) : Lattice<19>::w(i); }

// Template of one particle (section 2.2): digitised ball |o - phi| <= r, BS
// = ball sites linked (any lattice velocity) to a site outside the ball, IS =
// other ball sites linked to a BS site, interior = the remaining ball sites.
// Entries come kind by kind (BS, then IS, then interior), each kind in z, y,
// x order so that neighbouring threads of the sparse kernels touch
// neighbouring sites: the per-particle sums read the BS entries alone.
void build_template(int q, double r, const double phi[3], std::vector<int>& out, int* nbs, int* nis, int* nin) {
  const int dim = q == 9 ? 2 : 3;
  const int R = (int)std::ceil(r) + 1;
  const int h = R + 1, ext = 2 * R + 3;
  const int ez = dim == 3 ? ext : 1, hz = dim == 3 ? h : 0, Rz = dim == 3 ? R : 0;
  std::vector<char> in((size_t)ext * ext * ez, 0), bs(in.size(), 0), is(in.size(), 0);
  auto gi = [&](int x, int y, int z) { return ((size_t)(z + hz) * ext + (y + h)) * ext + (x + h); };
  int cx[19], cy[19], cz[19];
  for (int i = 0; i < q; i++) {
    cx[i] = q == 9 ? Lattice<9>::cx(i) : Lattice<19>::cx(i);
    cy[i] = q == 9 ? Lattice<9>::cy(i) : Lattice<19>::cy(i);
    cz[i] = q == 9 ? Lattice<9>::cz(i) : Lattice<19>::cz(i);
  }
  for (int z = -Rz; z <= Rz; z++)
    for (int y = -R; y <= R; y++)
      for (int x = -R; x <= R; x++) {
        const double dx = x - phi[0], dy = y - phi[1], dz = z - phi[2];
        in[gi(x, y, z)] = dx * dx + dy * dy + dz * dz <= r * r;
      }
  *nbs = *nis = *nin = 0;
  for (int z = -Rz; z <= Rz; z++)
    for (int y = -R; y <= R; y++)
      for (int x = -R; x <= R; x++) {
        if (!in[gi(x, y, z)]) continue;
        for (int i = 1; i < q; i++)
          if (!in[gi(x + cx[i], y + cy[i], z + cz[i])]) {
            bs[gi(x, y, z)] = 1;
            break;
          }
      }
  for (int z = -Rz; z <= Rz; z++)
    for (int y = -R; y <= R; y++)
      for (int x = -R; x <= R; x++) {
        if (!in[gi(x, y, z)] || bs[gi(x, y, z)]) continue;
        for (int i = 1; i < q; i++)
          if (bs[gi(x + cx[i], y + cy[i], z + cz[i])]) {
            is[gi(x, y, z)] = 1;
            break;
          }
      }
  for (int want = 1; want <= 3; want++)
    for (int z = -Rz; z <= Rz; z++)
      for (int y = -R; y <= R; y++)
        for (int x = -R; x <= R; x++) {
          const size_t g = gi(x, y, z);
          if (!in[g]) continue;
          const int kind = bs[g] ? 1 : (is[g] ? 2 : 3);
          if (kind != want) continue;
          out.push_back(pack_entry(x, y, z, kind));
          (kind == 1 ? *nbs : kind == 2 ? *nis : *nin) += 1;
        }
}

// The owner map of the current shifts, for read-outs: contexts with kind
// grids keep none between steps, so every site is emptied and every BS/IS
// entry claims its site again (lowest entry, hence lowest particle id).
int refresh_owner_map(lbm_ctx* c) {
  if (!c->grids) return LBM_OK;
  k_fill<int><<<blocks_for(c->NT), 256, 0, c->stream>>>(c->own, c->NT, kEmpty);
  if (c->nent > 0)
    k_stamp<<<blocks_for(c->nent), 256, 0, c->stream>>>(c->own, c->P, c->E, boxes_arg(c), 0, (int)c->nent);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

int check_status(lbm_ctx* c) {
  int st[4];
  HIP_TRY(hipMemcpyAsync(st, c->status, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (st[0] != 0) {
    const int zero[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(c->status, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (st[0] & kStatusRecord) return LBM_ESTATE;
    if (st[0] & kStatusCollision) return LBM_ECOLLISION;
    if (st[0] & kStatusClosure) return LBM_ECAPACITY;
  }
  return LBM_OK;
}

// Box table and per-box forcing terms 3 w_i c_i . f_b to the device.
int upload_boxes(lbm_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->d_boxes, c->boxes.data(), sizeof(Geo) * c->nbox, hipMemcpyHostToDevice, c->stream));
  std::vector<double> fd((size_t)c->nbox * c->q);
  for (int b = 0; b < c->nbox; b++)
    for (int i = 0; i < c->q; i++) {
      const int cx = c->q == 9 ? Lattice<9>::cx(i) : Lattice<19>::cx(i);
      const int cy = c->q == 9 ? Lattice<9>::cy(i) : Lattice<19>::cy(i);
      const int cz = c->q == 9 ? Lattice<9>::cz(i) : Lattice<19>::cz(i);
      const double cf = cx * c->fbb[3 * b] + cy * c->fbb[3 * b + 1] + cz * c->fbb[3 * b + 2];
      fd[(size_t)b * c->q + i] = 3.0 * lattice_w(c->q, i) * cf;
    }
  if (c->prm.storage == LBM_FP64) {
    HIP_TRY(hipMemcpyAsync(c->d_fbt, fd.data(), sizeof(double) * fd.size(), hipMemcpyHostToDevice, c->stream));
  } else {
    std::vector<float> ff(fd.begin(), fd.end());
    HIP_TRY(hipMemcpyAsync(c->d_fbt, ff.data(), sizeof(float) * ff.size(), hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));  // the host vectors die here
  return LBM_OK;
}

void drop_graph(lbm_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

template <typename V>
int upload(lbm_ctx* c, V* dst, const V* src, size_t count) {
  if (count == 0) return LBM_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, sizeof(V) * count, hipMemcpyHostToDevice, c->stream));
  return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free stepping (lbm_step_noalloc): the per-step scratch of the
// particle kernels -- per-particle momentum sums, close-pair and site-sharing
// lists, pair staging; each written by the step before it is read -- in one
// library array per device instead of the context's workspace.  The array is
// file scope, so every device holds its own copy at its own address: host
// code takes that address from hipGetSymbolAddress, once per device, and
// never uses the array's name as a device pointer.
// ---------------------------------------------------------------------------
namespace {

constexpr int kScratchParticles = 4096;
constexpr size_t scr_round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kScrDP = 0;
constexpr size_t kScrDL = kScrDP + scr_round(sizeof(double) * 3 * kScratchParticles);
constexpr size_t kScrCandN = kScrDL + scr_round(sizeof(double) * 3 * kScratchParticles);
constexpr size_t kScrCand = kScrCandN + scr_round(sizeof(int) * kScratchParticles);
constexpr size_t kScrPairs = kScrCand + scr_round(sizeof(int) * (size_t)kScratchParticles * kCandMax);
constexpr size_t kScrNbrN = kScrPairs + scr_round(sizeof(int) * 2 * (size_t)kScratchParticles * kCandMax);
constexpr size_t kScrNbr = kScrNbrN + scr_round(sizeof(int) * kScratchParticles);
constexpr size_t kScratchBytes = kScrNbr + scr_round(sizeof(int) * (size_t)kScratchParticles * kNbrMax);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the scratch array on device dev (the current device).
int scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return LBM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EHIP;
    g_scratch[dev] = ptr;
  }
  *out = (char*)g_scratch[dev];
  return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int lbm_workspace_size(const lbm_params* prm, size_t* bytes) {
  const int rc = check_params(prm);
  if (rc != LBM_OK) return rc;
  if (!bytes) return LBM_EINVAL;
  const int32_t dims[3] = {prm->nx, prm->ny, prm->nz};
  *bytes = make_layout(*prm, make_boxset(1, dims)).total;
  return LBM_OK;
}

int lbm_ensemble_workspace_size(const lbm_params* prm, int32_t nbox, const int32_t* dims, size_t* bytes) {
  const int rc = check_boxes(prm, nbox, dims);
  if (rc != LBM_OK) return rc;
  if (!bytes) return LBM_EINVAL;
  *bytes = make_layout(*prm, make_boxset(nbox, dims)).total;
  return LBM_OK;
}

int lbm_bytes_per_site(const lbm_params* prm, int64_t* bytes) {
  if (!prm || !bytes) return LBM_EINVAL;
  if (prm->lattice != LBM_D2Q9 && prm->lattice != LBM_D3Q19) return LBM_EINVAL;
  *bytes = 2 * (int64_t)prm->lattice * (int64_t)store_size(prm->storage);
  return LBM_OK;
}

static int create_impl(const lbm_params* prm, int nbox, const int32_t* dims, void* d_workspace, size_t bytes,
                       void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  const BoxSet bset = make_boxset(nbox, dims);
  const Layout L = make_layout(*prm, bset);
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0 || bytes < L.total) return LBM_EWORKSPACE;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_EINVAL;
  c->prm = *prm;
  c->q = prm->lattice;
  c->dim = prm->lattice == LBM_D2Q9 ? 2 : 3;
  c->nbox = nbox;
  c->NT = bset.NT;
  c->PS = pop_stride(bset.NT);
  int64_t off = 0;
  for (int b = 0; b < nbox; b++) {
    const int nx = dims[3 * b], ny = dims[3 * b + 1], nz = dims[3 * b + 2];
    const int64_t N = (int64_t)nx * ny * nz;
    c->boxes.push_back(Geo{nx, ny, nz, N, prm->walls, off, 0});
    off += N;
  }
  c->G = c->boxes[0];
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_workspace;
  c->L = L;
  c->f[0] = c->ws + L.f[0];
  c->f[1] = c->ws + L.f[1];
  c->cur = 0;
  c->drho = c->ws + L.drho;
  c->slot = (double*)(c->ws + L.slot);
  c->vel = c->ws + L.vel;
  c->own = (int*)(c->ws + L.own);
  c->flag = (uint8_t*)(c->ws + L.flag);
  c->status = (int*)(c->ws + L.status);
  c->d_boxes = (Geo*)(c->ws + L.boxes);
  c->d_fbt = c->ws + L.fbt;
  c->d_tiles = (int4*)(c->ws + L.tiles);
  c->ntiles = 0;
  c->tiles_w = 0;
  {
    int dev = 0, gy = 0, gz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&gy, hipDeviceAttributeMaxGridDimY, dev) != hipSuccess ||
        hipDeviceGetAttribute(&gz, hipDeviceAttributeMaxGridDimZ, dev) != hipSuccess) {
      delete c;
      return LBM_EHIP;
    }
    c->row_ok = nbox == 1 && dims[1] <= gy && dims[2] <= gz;
    c->device = dev;
  }
  // one box: the row kernel; an ensemble: tiles of 128 sites, one workgroup each
  c->sweep_w = c->row_ok ? 0 : 128;
  c->sweep_grid = 0;
  c->sweep_occ = 0;
  c->cap = nullptr;
  c->graph = nullptr;
  c->gexec = nullptr;
  c->graph_steps = 0;
  char* w = c->ws;
  c->P = DevParticles{(double*)(w + L.x),    (double*)(w + L.x0),  (double*)(w + L.u),
                      (double*)(w + L.om),   (double*)(w + L.phi), (double*)(w + L.fext),
                      (double*)(w + L.dP),   (double*)(w + L.dL),  (double*)(w + L.F),
                      (double*)(w + L.T),    (double*)(w + L.m),   (double*)(w + L.I),
                      (double*)(w + L.rad),  (int*)(w + L.b0),     (int*)(w + L.k),
                      (int*)(w + L.org),
                      (int*)(w + L.ent0),    (int*)(w + L.nbs),    (int*)(w + L.nis),
                      (int*)(w + L.nin),     (int*)(w + L.cand_n), (int*)(w + L.jump),
                      (int*)(w + L.box),     (double*)(w + L.fc),
                      (int*)(w + L.cand),    (int*)(w + L.pairs),
                      (int*)(w + L.orgp),    (int*)(w + L.moved),
                      (int*)(w + L.kg0),     (int*)(w + L.kgR),
                      (int*)(w + L.nbr_n),   (int*)(w + L.nbr),
                      (uint8_t*)(w + L.kgrid)};
  c->d_clo = (float*)(w + L.clo);
  c->closure = 0;
  c->clo_h = 0.0;
  c->E = DevEntries{(int*)(w + L.off), (int*)(w + L.pid)};
  c->np = 0;
  c->nent = 0;
  c->fbb.assign(3 * (size_t)nbox, 0.0);
  for (int b = 0; b < nbox; b++)
    for (int a = 0; a < 3; a++) c->fbb[3 * b + a] = prm->body_force[a];
  c->prof = false;
  c->failed = false;
  c->ev_used = 0;
  {
    // one workgroup per particle while the largest ball's bounding box, (2 floor(r + 1/2)
    // + 1)^d sites and so a bound on its entries, stays within kPrepareLocalMax; larger
    // balls spread their entries over the grid
    c->grids = uses_kind_grids(c->dim, prm->max_radius);
    c->kg_used = 0;
    // about one workgroup per kPrepareBlock entries of the largest ball (its
    // volume), so that a particle's scattered IS stores spread over CUs
    const double r = prm->max_radius;
    const double vol = c->dim == 3 ? 4.0 / 3.0 * M_PI * r * r * r : M_PI * r * r;
    c->prep_split = std::max(1, std::min(8, (int)std::ceil(vol / kPrepareBlock)));
    c->small_ball = vol <= kSmallBall;
  }
  // fluid at rest: every deviation zero; empty map; clear status
  const size_t fbytes = (size_t)c->q * c->PS * store_size(prm->storage);
  const int64_t nwords = (int64_t)(fbytes / 4);
  k_fill<uint32_t><<<blocks_for(nwords), 256, 0, c->stream>>>((uint32_t*)c->f[0], nwords, 0u);
  k_fill<int><<<blocks_for(c->NT), 256, 0, c->stream>>>(c->own, c->NT, kEmpty);
  k_fill<uint8_t><<<blocks_for(c->NT), 256, 0, c->stream>>>(c->flag, c->NT, (uint8_t)0);
  k_fill<int><<<1, 256, 0, c->stream>>>(c->status, 16, 0);
  if (prm->storage == LBM_FP64)
    k_fill_records<double><<<blocks_for(c->NT), 256, 0, c->stream>>>((double*)c->vel, c->NT);
  else
    k_fill_records<float><<<blocks_for(c->NT), 256, 0, c->stream>>>((float*)c->vel, c->NT);
  if (hipGetLastError() != hipSuccess || upload_boxes(c) != LBM_OK ||
      (tile_width(c->sweep_w) && build_tiles(c, c->sweep_w) != LBM_OK) ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return LBM_EHIP;
  }
  *out = c;
  return LBM_OK;
}

int lbm_create(const lbm_params* prm, void* d_workspace, size_t bytes, void* hip_stream, lbm_ctx** out) {
  const int rc = check_params(prm);
  if (rc != LBM_OK) return rc;
  const int32_t dims[3] = {prm->nx, prm->ny, prm->nz};
  return create_impl(prm, 1, dims, d_workspace, bytes, hip_stream, out);
}

int lbm_ensemble_create(const lbm_params* prm, int32_t nbox, const int32_t* dims, void* d_workspace, size_t bytes,
                        void* hip_stream, lbm_ctx** out) {
  const int rc = check_boxes(prm, nbox, dims);
  if (rc != LBM_OK) return rc;
  return create_impl(prm, nbox, dims, d_workspace, bytes, hip_stream, out);
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  drop_graph(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return LBM_OK;
}

static int add_impl(lbm_ctx* c, int32_t bx, int32_t n, const double* x, const double* u, const double* omega,
                    const double* radius, const double* mass, const double* inertia, int32_t* first_id) {
  if (!c || n < 0 || bx < 0 || bx >= c->nbox) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  // particles of a box have consecutive ids: boxes are filled in order
  if (c->np > 0 && bx < c->h_box.back()) return LBM_EINVAL;
  if (n == 0) {
    if (first_id) *first_id = c->np;
    return LBM_OK;
  }
  if (!x || !radius || !mass || !inertia) return LBM_EINVAL;
  if (c->np + (int64_t)n > c->prm.max_particles) return LBM_ECAPACITY;
  const int dim = c->dim;
  const Geo& BG = c->boxes[bx];
  const int box[3] = {BG.nx, BG.ny, BG.nz};
  for (int j = 0; j < n; j++) {
    for (int a = 0; a < 3; a++) {
      if (a < dim && !std::isfinite(x[3 * j + a])) return LBM_ENONFINITE;
      if (u && a < dim && !std::isfinite(u[3 * j + a])) return LBM_ENONFINITE;
      if (omega && !std::isfinite(omega[3 * j + a])) return LBM_ENONFINITE;
      if (a < dim && (x[3 * j + a] < 0 || x[3 * j + a] >= box[a])) return LBM_EINVAL;
    }
    const double r = radius[j];
    if (!std::isfinite(r) || std::isnan(mass[j]) || std::isnan(inertia[j])) return LBM_ENONFINITE;
    if (!(r > 0) || r > c->prm.max_radius) return LBM_EINVAL;
    if (!(mass[j] > 0) || !(inertia[j] > 0)) return LBM_EINVAL;
    for (int a = 0; a < dim; a++)
      if (2 * (int)std::ceil(r) + 3 > box[a]) return LBM_EINVAL;
    for (int a = 0; a < dim; a++)
      if (((c->prm.walls >> a) & 1) && (x[3 * j + a] - r < 1.0 || x[3 * j + a] + r > box[a] - 2.0))
        return LBM_EOVERLAP;
  }
  // positions of the particles already in the box
  std::vector<double> cur((size_t)3 * c->np);
  if (c->np > 0) {
    HIP_TRY(hipMemcpyAsync(cur.data(), c->P.x, sizeof(double) * 3 * c->np, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  auto dist2 = [&](const double* A, const double* B) {
    double s = 0;
    for (int a = 0; a < dim; a++) {
      double d = B[a] - A[a];
      d -= box[a] * std::floor(d / box[a] + 0.5);
      s += d * d;
    }
    return s;
  };
  for (int j = 0; j < n; j++) {
    for (int p = 0; p < c->np; p++) {
      if (c->h_box[p] != bx) continue;  // boxes are independent
      const double lim = radius[j] + c->h_rad[p];
      if (dist2(&cur[3 * p], &x[3 * j]) < lim * lim) return LBM_EOVERLAP;
    }
    for (int i = 0; i < j; i++) {
      const double lim = radius[j] + radius[i];
      if (dist2(&x[3 * i], &x[3 * j]) < lim * lim) return LBM_EOVERLAP;
    }
  }
  // templates and particle records (host), then upload
  std::vector<double> hx(3 * n), hu(3 * n, 0.0), hom(3 * n, 0.0), hphi(3 * n), hfext(3 * n);
  std::vector<int> hb0(3 * n), hk(3 * n, 0), hent0(n), hnbs(n), hnis(n), hnin(n), hoff, hpid;
  for (int j = 0; j < n; j++) {
    const double r = radius[j];
    const double V = dim == 2 ? M_PI * r * r : 4.0 / 3.0 * M_PI * r * r * r;
    for (int a = 0; a < 3; a++) {
      hx[3 * j + a] = a < dim ? x[3 * j + a] : 0.0;
      if (u && a < dim) hu[3 * j + a] = u[3 * j + a];
      if (omega && (dim == 3 || a == 2)) hom[3 * j + a] = omega[3 * j + a];
      hb0[3 * j + a] = (int)std::floor(hx[3 * j + a] + 0.5);
      hphi[3 * j + a] = hx[3 * j + a] - (double)hb0[3 * j + a];
      hfext[3 * j + a] = std::isinf(mass[j]) ? 0.0 : (mass[j] - c->prm.rho0 * V) * c->prm.gravity[a];
    }
    int nb = 0, ni = 0, nn = 0;
    const size_t before = hoff.size();
    build_template(c->q, r, &hphi[3 * j], hoff, &nb, &ni, &nn);
    hent0[j] = (int)(c->nent + before);
    hnbs[j] = nb;
    hnis[j] = ni;
    hnin[j] = nn;
    hpid.insert(hpid.end(), (size_t)(nb + ni + nn), c->np + j);
  }
  if (c->nent + (int64_t)hoff.size() > c->L.max_ent) return LBM_ECAPACITY;
  // Kind grids of the new particles and the lists of particles that may share
  // a site (the box's particles, old and new, within r_i + r_j + kShareMargin)
  std::vector<uint8_t> hkg;
  std::vector<int> hkg0(n), hkgR(n), hnbr_n, hnbr;
  int pbox0 = c->np;  // first particle of box bx
  while (pbox0 > 0 && c->h_box[pbox0 - 1] == bx) pbox0--;
  if (c->grids) {
    size_t at = c->kg_used;
    for (int j = 0; j < n; j++) {
      const int R = kind_grid_half(radius[j]), W = 2 * R + 1;
      const size_t nb = dim == 2 ? (size_t)W * W : (size_t)W * W * W;
      const size_t g0 = hkg.size();
      hkg.resize(g0 + nb, 0);
      const int eb = hent0[j] - (int)c->nent, ee = eb + hnbs[j] + hnis[j] + hnin[j];
      for (int e = eb; e < ee; e++) {
        const int v = hoff[e];
        const int ox = (int)(int8_t)(v & 0xff), oy = (int)(int8_t)((v >> 8) & 0xff), oz = (int)(int8_t)((v >> 16) & 0xff);
        if (std::abs(ox) > R || std::abs(oy) > R || std::abs(oz) > R) return LBM_EINVAL;  // cannot happen
        const size_t idx = dim == 2 ? (size_t)(oy + R) * W + (ox + R) : ((size_t)(oz + R) * W + (oy + R)) * W + (ox + R);
        hkg[g0 + idx] = (uint8_t)entry_kind(v);
      }
      hkg0[j] = (int)(at + g0);
      hkgR[j] = R;
    }
    const int nb_all = c->np + n - pbox0;
    hnbr_n.assign(nb_all, 0);
    hnbr.assign((size_t)nb_all * kNbrMax, 0);
    auto pos = [&](int q) { return q < c->np ? &cur[3 * q] : &x[3 * (q - c->np)]; };
    auto rad = [&](int q) { return q < c->np ? c->h_rad[q] : radius[q - c->np]; };
    for (int a = pbox0; a < c->np + n; a++)
      for (int b = pbox0; b < c->np + n; b++) {
        if (a == b) continue;
        const double lim = rad(a) + rad(b) + kShareMargin;
        if (dist2(pos(a), pos(b)) > lim * lim) continue;
        int& cnt = hnbr_n[a - pbox0];
        if (cnt >= kNbrMax) return LBM_ECAPACITY;
        hnbr[(size_t)(a - pbox0) * kNbrMax + cnt++] = b;
      }
  }
  // Every argument has been checked: from here on only a HIP error can fail
  // the call.  The host bookkeeping is then put back as it was, and the
  // context is marked failed (the device map may already hold stamps of the
  // rejected particles), so that every later call reports LBM_EHIP.
  const int p0 = c->np;
  const int64_t e0 = c->nent, e1 = c->nent + (int64_t)hoff.size();
  const std::vector<Geo> boxes_before = c->boxes;
  const std::vector<double> fbb_before = c->fbb;
  auto fail = [&](int code) {
    c->boxes = boxes_before;
    c->G = c->boxes[0];
    c->fbb = fbb_before;
    c->np = p0;
    c->nent = e0;
    c->failed = true;
    return code;
  };
  int rc;
#define UP(dst, src, cnt) \
  if ((rc = upload(c, dst, src, cnt)) != LBM_OK) return fail(rc)
  UP(c->P.x + 3 * p0, hx.data(), 3 * (size_t)n);
  UP(c->P.x0 + 3 * p0, hx.data(), 3 * (size_t)n);
  UP(c->P.u + 3 * p0, hu.data(), 3 * (size_t)n);
  UP(c->P.om + 3 * p0, hom.data(), 3 * (size_t)n);
  UP(c->P.phi + 3 * p0, hphi.data(), 3 * (size_t)n);
  UP(c->P.fext + 3 * p0, hfext.data(), 3 * (size_t)n);
  UP(c->P.m + p0, mass, (size_t)n);
  UP(c->P.I + p0, inertia, (size_t)n);
  UP(c->P.rad + p0, radius, (size_t)n);
  UP(c->P.b0 + 3 * p0, hb0.data(), 3 * (size_t)n);
  UP(c->P.k + 3 * p0, hk.data(), 3 * (size_t)n);
  std::vector<int> horg(3 * n);
  for (int j = 0; j < n; j++)
    for (int a = 0; a < 3; a++) horg[3 * j + a] = ((hb0[3 * j + a] % box[a]) + box[a]) % box[a];
  UP(c->P.org + 3 * p0, horg.data(), 3 * (size_t)n);
  UP(c->P.ent0 + p0, hent0.data(), (size_t)n);
  UP(c->P.nbs + p0, hnbs.data(), (size_t)n);
  UP(c->P.nis + p0, hnis.data(), (size_t)n);
  UP(c->P.nin + p0, hnin.data(), (size_t)n);
  const std::vector<int> hbox((size_t)n, bx);
  UP(c->P.box + p0, hbox.data(), (size_t)n);
  UP(c->E.off + c->nent, hoff.data(), hoff.size());
  UP(c->E.pid + c->nent, hpid.data(), hpid.size());
  const std::vector<double> zero(3 * (size_t)n, 0.0);
  UP(c->P.F + 3 * p0, zero.data(), 3 * (size_t)n);
  UP(c->P.T + 3 * p0, zero.data(), 3 * (size_t)n);
  UP(c->P.fc + 3 * p0, zero.data(), 3 * (size_t)n);
  UP(c->P.orgp + 3 * p0, horg.data(), 3 * (size_t)n);
  const std::vector<int> izero((size_t)n, 0);
  UP(c->P.moved + p0, izero.data(), (size_t)n);
  UP(c->P.jump + p0, izero.data(), (size_t)n);
  if (c->grids) {
    UP(c->P.kgrid + c->kg_used, hkg.data(), hkg.size());
    UP(c->P.kg0 + p0, hkg0.data(), (size_t)n);
    UP(c->P.kgR + p0, hkgR.data(), (size_t)n);
    UP(c->P.nbr_n + pbox0, hnbr_n.data(), hnbr_n.size());
    UP(c->P.nbr + (size_t)pbox0 * kNbrMax, hnbr.data(), hnbr.size());
  }
#undef UP
  // stamp the new entries into the current map (existing owners have lower ids)
  for (int b = bx; b < c->nbox; b++) c->boxes[b].p1 = c->np + n;  // later boxes are still empty
  c->G = c->boxes[0];
  if (e1 > e0 && !c->grids) {  // particles this small may hold no site at all
    k_stamp<<<blocks_for(e1 - e0), 256, 0, c->stream>>>(c->own, c->P, c->E, boxes_arg(c), (int)e0, (int)e1);
    if (hipGetLastError() != hipSuccess) return fail(LBM_EHIP);
  }
  c->nent = e1;
  c->np += n;
  // flags and records of every ball site, with nothing pending
  const int prc = DISPATCH(c, launch_prepare, c, 0, 1);
  if (prc != LBM_OK) return fail(prc);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(LBM_EHIP);
  // fluid body force of every box: user value, plus the opposite of the
  // box's particles' total external force spread over its sites in a
  // zero-net-force box
  std::vector<double> tot(3 * (size_t)c->nbox, 0.0);
  for (int p = 0; p < p0; p++)
    for (int a = 0; a < 3; a++) tot[3 * c->h_box[p] + a] += c->h_fext[3 * p + a];
  for (int j = 0; j < n; j++)
    for (int a = 0; a < 3; a++) tot[3 * bx + a] += hfext[3 * j + a];
  for (int b = 0; b < c->nbox; b++)
    for (int a = 0; a < 3; a++)
      c->fbb[3 * b + a] =
          c->prm.body_force[a] - (c->prm.zero_net_force ? tot[3 * b + a] / (double)c->boxes[b].N : 0.0);
  if (upload_boxes(c) != LBM_OK) return fail(LBM_EHIP);
  // the call has succeeded: the host copies of the particle set grow
  c->kg_used += hkg.size();
  for (int j = 0; j < n; j++) {
    c->h_x0.insert(c->h_x0.end(), &hx[3 * j], &hx[3 * j] + 3);
    c->h_rad.push_back(radius[j]);
    c->h_m.push_back(mass[j]);
    c->h_I.push_back(inertia[j]);
    c->h_fext.insert(c->h_fext.end(), &hfext[3 * j], &hfext[3 * j] + 3);
    c->h_nbs.push_back(hnbs[j]);
    c->h_nis.push_back(hnis[j]);
    c->h_nin.push_back(hnin[j]);
  }
  c->h_off.insert(c->h_off.end(), hoff.begin(), hoff.end());
  c->h_pid.insert(c->h_pid.end(), hpid.begin(), hpid.end());
  c->h_box.insert(c->h_box.end(), (size_t)n, bx);
  drop_graph(c);
  if (first_id) *first_id = p0;
  return LBM_OK;
}

int lbm_add_particles(lbm_ctx* c, int32_t n, const double* x, const double* u, const double* omega,
                      const double* radius, const double* mass, const double* inertia, int32_t* first_id) {
  return add_impl(c, 0, n, x, u, omega, radius, mass, inertia, first_id);
}

int lbm_ensemble_add_particles(lbm_ctx* c, int32_t box, int32_t n, const double* x, const double* u,
                               const double* omega, const double* radius, const double* mass,
                               const double* inertia, int32_t* first_id) {
  return add_impl(c, box, n, x, u, omega, radius, mass, inertia, first_id);
}

// Capture graph_steps steps (an even number, so the population buffers come
// back to the same roles) on a private stream; the graph is rebuilt when the
// particle set, the buffer roles or the sweep launch shape changed.
static int ensure_graph(lbm_ctx* c) {
  if (c->gexec && c->g_steps == c->graph_steps && c->g_cur == c->cur && c->g_np == c->np &&
      c->g_nent == c->nent && c->g_w == c->sweep_w && c->g_grid == c->sweep_grid && c->g_occ == c->sweep_occ)
    return LBM_OK;
  drop_graph(c);
  if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  const bool prof = c->prof;
  const int cur0 = c->cur;
  c->stream = c->cap;
  c->prof = false;
  int rc = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) == hipSuccess ? LBM_OK : LBM_EHIP;
  for (int t = 0; rc == LBM_OK && t < c->graph_steps; t++) rc = DISPATCH(c, launch_step, c);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->cap, &g);
  c->stream = user;
  c->prof = prof;
  c->cur = cur0;  // nothing ran yet
  if (rc != LBM_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return LBM_EHIP;
  }
  c->graph = g;
  if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(c);
    return LBM_EHIP;
  }
  c->g_steps = c->graph_steps;
  c->g_cur = c->cur;
  c->g_np = c->np;
  c->g_nent = c->nent;
  c->g_w = c->sweep_w;
  c->g_grid = c->sweep_grid;
  c->g_occ = c->sweep_occ;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  if (tile_width(c->sweep_w)) {
    const int rc = build_tiles(c, c->sweep_w);
    if (rc != LBM_OK) return rc;
  }
  if (c->graph_steps > 0) {
    while (nsteps >= c->graph_steps) {
      const int rc = ensure_graph(c);
      if (rc != LBM_OK) return rc;
      HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
      nsteps -= c->graph_steps;
    }
  }
  for (int t = 0; t < nsteps; t++) {
    const int rc = DISPATCH(c, launch_step, c);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int lbm_step_noalloc(lbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  if (c->np > kScratchParticles) return LBM_ECAPACITY;
  // the tiles of a tile-kernel shape are built by the call that set it
  if (tile_width(c->sweep_w) && c->tiles_w != c->sweep_w) return LBM_EINVAL;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device) return LBM_EINVAL;
  char* sp = nullptr;
  const int arc = scratch_address(dev, &sp);
  if (arc != LBM_OK) return arc;
  // the same launches as lbm_step, eager and without profiling events, on
  // the particle arrays with their per-step scratch in the library array
  const DevParticles keep = c->P;
  const bool prof = c->prof;
  c->P.dP = (double*)(sp + kScrDP);
  c->P.dL = (double*)(sp + kScrDL);
  c->P.cand_n = (int*)(sp + kScrCandN);
  c->P.cand = (int*)(sp + kScrCand);
  c->P.pairs = (int*)(sp + kScrPairs);
  c->P.nbr_n = (int*)(sp + kScrNbrN);
  c->P.nbr = (int*)(sp + kScrNbr);
  c->prof = false;
  int rc = LBM_OK;
  for (int t = 0; t < nsteps && rc == LBM_OK; t++) rc = DISPATCH(c, launch_step, c);
  c->P = keep;
  c->prof = prof;
  return rc;
}

int lbm_set_graph(lbm_ctx* c, int32_t steps_per_graph) {
  if (!c || steps_per_graph < 0 || steps_per_graph % 2) return LBM_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->graph_steps = steps_per_graph;
  drop_graph(c);
  return LBM_OK;
}

int lbm_set_sweep_config(lbm_ctx* c, int32_t width, int32_t grid, int32_t blocks_per_cu) {
  if (!c || grid < 0 || !occ_ok(c, blocks_per_cu)) return LBM_EINVAL;
  if (width != 0 && !tile_width(width)) return LBM_EINVAL;
  if (width == 0 && !c->row_ok) return LBM_EINVAL;  // the row kernel covers one box
  if (tile_width(width)) {
    const int rc = build_tiles(c, width);
    if (rc != LBM_OK) return rc;
  }
  c->sweep_w = width;
  c->sweep_grid = tile_width(width) ? grid : 0;
  c->sweep_occ = blocks_per_cu;
  return LBM_OK;
}

int lbm_get_sweep_config(lbm_ctx* c, int32_t* width, int32_t* grid, int32_t* blocks_per_cu) {
  if (!c) return LBM_EINVAL;
  if (width) *width = c->sweep_w;
  if (grid) *grid = c->sweep_grid;
  if (blocks_per_cu) *blocks_per_cu = c->sweep_occ;
  return LBM_OK;
}

// The sweep launches both tuners try: shapes x occupancy caps (fewer
// resident waves can stream faster).
struct SweepCand {
  int w, g, occ;
};
static std::vector<SweepCand> sweep_candidates(const lbm_ctx* c, int ncu) {
  std::vector<SweepCand> cands;
  for (int occ : {0, 6, 5, 4, 3, 2}) {
    if (!occ_ok(c, occ)) continue;
    if (c->row_ok) cands.push_back({0, 0, occ});
    for (int w : {64, 128, 256, 512})
      for (int k : {0, 4, 8, 16, 32}) cands.push_back({w, k * ncu, occ});
  }
  return cands;
}

int lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* width, int32_t* grid, int32_t* blocks_per_cu,
                 double* best_ms) {
  if (!c || reps < 1) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  if (c->prm.aa) return LBM_EINVAL;  // a sweep in place cannot be repeated on the live state
  // a sweep recomputes B and the ball-site scratch from A and the records,
  // so repeating it leaves the state as one sweep does: time the candidates
  // on the live state
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const std::vector<SweepCand> cands = sweep_candidates(c, ncu);
  using Cand = SweepCand;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = LBM_OK;
  // time `n` sweeps of one candidate (after one untimed), in ms per sweep
  auto time_cand = [&](const Cand& cd, int n, double& ms_out) {
    if (tile_width(cd.w) && (rc = build_tiles(c, cd.w)) != LBM_OK) return false;
    if ((rc = DISPATCH(c, launch_sweep, c, cd.w, cd.g, cd.occ)) != LBM_OK) return false;  // warm-up
    if (hipEventRecord(e0, c->stream) != hipSuccess) {
      rc = LBM_EHIP;
      return false;
    }
    for (int r = 0; r < n && rc == LBM_OK; r++) rc = DISPATCH(c, launch_sweep, c, cd.w, cd.g, cd.occ);
    if (rc != LBM_OK) return false;
    float ms = 0;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = LBM_EHIP;
      return false;
    }
    ms_out = ms / n;
    return true;
  };
  // every candidate once, then the four fastest again in two alternating
  // rounds of twice the sweeps (a single short timing misranks candidates
  // within a few per cent of each other)
  std::vector<std::pair<double, int>> first;
  for (size_t k = 0; k < cands.size(); k++) {
    double ms = 0;
    if (!time_cand(cands[k], reps, ms)) break;
    first.push_back({ms, (int)k});
  }
  double best = 1e300;
  Cand win = {c->sweep_w, c->sweep_grid, c->sweep_occ};
  if (rc == LBM_OK) {
    std::sort(first.begin(), first.end());
    const size_t top = std::min<size_t>(4, first.size());
    std::vector<double> sum(top, 0.0);
    for (int round = 0; round < 2 && rc == LBM_OK; round++)
      for (size_t t = 0; t < top; t++) {
        double ms = 0;
        if (!time_cand(cands[first[t].second], 2 * reps, ms)) break;
        sum[t] += ms;
      }
    for (size_t t = 0; t < top && rc == LBM_OK; t++)
      if (sum[t] / 2 < best) {
        best = sum[t] / 2;
        win = cands[first[t].second];
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LBM_OK) return rc;
  rc = lbm_set_sweep_config(c, win.w, win.g, win.occ);
  if (rc != LBM_OK) return rc;
  if (width) *width = win.w;
  if (grid) *grid = win.g;
  if (blocks_per_cu) *blocks_per_cu = win.occ;
  if (best_ms) *best_ms = best;
  return LBM_OK;
}

int lbm_autotune_steps(lbm_ctx* c, int32_t steps, int32_t* width, int32_t* grid, int32_t* blocks_per_cu,
                       double* best_ms, int64_t* steps_done) {
  if (!c || steps < 1) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const std::vector<SweepCand> cands = sweep_candidates(c, ncu);
  // whole steps, an even number so that both halves of the AA pattern and
  // both buffer roles count alike; with step graphs set, whole graphs (short
  // steps launched one by one can be bound by the host's launch rate)
  const int gs = c->graph_steps;
  const int n1 = gs > 0 ? (steps + gs - 1) / gs * gs : steps + (steps & 1);
  const int warm = gs > 0 ? gs : 2;
  const bool prof = c->prof;
  c->prof = false;
  c->ev_used = 0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = LBM_OK;
  int64_t done = 0;
  auto time_cand = [&](const SweepCand& cd, int n, double& ms_out) {
    if ((rc = lbm_set_sweep_config(c, cd.w, cd.g, cd.occ)) != LBM_OK) return false;
    if ((rc = lbm_step(c, warm)) != LBM_OK) return false;  // untimed (captures a graph when set)
    done += warm;
    if (hipEventRecord(e0, c->stream) != hipSuccess) {
      rc = LBM_EHIP;
      return false;
    }
    if ((rc = lbm_step(c, n)) != LBM_OK) return false;
    done += n;
    float ms = 0;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = LBM_EHIP;
      return false;
    }
    ms_out = ms / n;
    return true;
  };
  // every candidate once, then the four fastest again in two alternating
  // rounds of twice the steps
  std::vector<std::pair<double, int>> first;
  for (size_t k = 0; k < cands.size(); k++) {
    double ms = 0;
    if (!time_cand(cands[k], n1, ms)) break;
    first.push_back({ms, (int)k});
  }
  double best = 1e300;
  SweepCand win = {c->sweep_w, c->sweep_grid, c->sweep_occ};
  if (rc == LBM_OK) {
    std::sort(first.begin(), first.end());
    const size_t top = std::min<size_t>(4, first.size());
    std::vector<double> sum(top, 0.0);
    for (int round = 0; round < 2 && rc == LBM_OK; round++)
      for (size_t t = 0; t < top; t++) {
        double ms = 0;
        if (!time_cand(cands[first[t].second], 2 * n1, ms)) break;
        sum[t] += ms;
      }
    for (size_t t = 0; t < top && rc == LBM_OK; t++)
      if (sum[t] / 2 < best) {
        best = sum[t] / 2;
        win = cands[first[t].second];
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->prof = prof;
  if (steps_done) *steps_done = done;
  if (rc != LBM_OK) return rc;
  rc = lbm_set_sweep_config(c, win.w, win.g, win.occ);
  if (rc != LBM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (width) *width = win.w;
  if (grid) *grid = win.g;
  if (blocks_per_cu) *blocks_per_cu = win.occ;
  if (best_ms) *best_ms = best;
  return check_status(c);
}

int lbm_set_closure(lbm_ctx* c, const float* d_params, double h_max) {
  if (!c || !std::isfinite(h_max) || h_max < 0) return LBM_EINVAL;
  if (c->dim != 2) return LBM_EUNSUPPORTED;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->closure = d_params != nullptr && h_max > 0;
  c->clo_h = h_max;
  if (d_params)
    HIP_TRY(hipMemcpyAsync(c->d_clo, d_params, sizeof(float) * mlp::kParams, hipMemcpyDeviceToDevice, c->stream));
  if (!c->closure && c->np > 0)
    k_fill<double><<<blocks_for(3 * (int64_t)c->np), 256, 0, c->stream>>>(c->P.fc, 3 * (int64_t)c->np, 0.0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_graph(c);
  return LBM_OK;
}

int lbm_closure_inputs(int32_t n, const double* xi, const double* d, const double* ri, const double* rj, double tau,
                       float* out) {
  if (n < 0 || (n > 0 && (!xi || !d || !ri || !rj || !out))) return LBM_EINVAL;
  for (int32_t k = 0; k < n; k++) mlp::closure_inputs(xi[2 * k], xi[2 * k + 1], ri[k], rj[k], d[2 * k], d[2 * k + 1],
                                                     tau, out + 8 * (size_t)k);
  return LBM_OK;
}

int lbm_box_info(lbm_ctx* c, int32_t box, int32_t* dims, int64_t* first_site, int32_t* first_particle,
                 int32_t* n_particles) {
  if (!c || box < 0 || box >= c->nbox) return LBM_EINVAL;
  const Geo& g = c->boxes[box];
  if (dims) {
    dims[0] = g.nx;
    dims[1] = g.ny;
    dims[2] = g.nz;
  }
  if (first_site) *first_site = g.off;
  int p0 = 0, cnt = 0;
  for (int p = 0; p < c->np; p++) {
    if (c->h_box[p] < box) p0 = p + 1;
    if (c->h_box[p] == box) cnt++;
  }
  if (first_particle) *first_particle = p0;
  if (n_particles) *n_particles = cnt;
  return LBM_OK;
}

int lbm_forces(lbm_ctx* c, double* F, double* T, double* x, double* u, double* omega) {
  if (!c) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  const size_t b = sizeof(double) * 3 * c->np;
  if (c->np > 0) {
    if (F) HIP_TRY(hipMemcpyAsync(F, c->P.F, b, hipMemcpyDeviceToHost, c->stream));
    if (T) HIP_TRY(hipMemcpyAsync(T, c->P.T, b, hipMemcpyDeviceToHost, c->stream));
    if (x) HIP_TRY(hipMemcpyAsync(x, c->P.x, b, hipMemcpyDeviceToHost, c->stream));
    if (u) HIP_TRY(hipMemcpyAsync(u, c->P.u, b, hipMemcpyDeviceToHost, c->stream));
    if (omega) HIP_TRY(hipMemcpyAsync(omega, c->P.om, b, hipMemcpyDeviceToHost, c->stream));
  }
  return check_status(c);
}

int lbm_fields(lbm_ctx* c, double* rho, double* u, int32_t* owner) {
  if (!c) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  if (rho || u) {
    // two arrays: the idle one stages the moments; AA: the staging area
    const size_t stage = c->prm.aa ? 4 * sizeof(double) * (size_t)std::min<int64_t>(c->NT, (int64_t)1 << 20)
                                   : (size_t)c->q * c->PS * store_size(c->prm.storage);
    const int64_t chunk = (int64_t)(stage / (4 * sizeof(double)));
    double* d_rho = c->prm.aa ? (double*)(c->ws + c->L.stage) : (double*)c->f[1 - c->cur];
    double* d_u = d_rho + chunk;
    for (int b = 0; b < c->nbox; b++) {
      const Geo& g = c->boxes[b];
      for (int64_t s0 = 0; s0 < g.N; s0 += chunk) {
        const int64_t cnt = std::min<int64_t>(chunk, g.N - s0);
        const int rc = DISPATCH(c, launch_moments, c, b, d_rho, d_u, s0, cnt);
        if (rc != LBM_OK) return rc;
        if (rho)
          HIP_TRY(hipMemcpyAsync(rho + g.off + s0, d_rho, sizeof(double) * cnt, hipMemcpyDeviceToHost, c->stream));
        if (u)
          HIP_TRY(hipMemcpyAsync(u + 3 * (g.off + s0), d_u, sizeof(double) * 3 * cnt, hipMemcpyDeviceToHost,
                                 c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
      }
    }
  }
  if (owner) {
    const int orc = refresh_owner_map(c);
    if (orc != LBM_OK) return orc;
    std::vector<int> m(c->NT);
    HIP_TRY(hipMemcpyAsync(m.data(), c->own, sizeof(int) * c->NT, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int64_t s = 0; s < c->NT; s++) owner[s] = m[s] == kEmpty ? -1 : c->h_pid[m[s] >> 1];
  }
  return check_status(c);
}

int lbm_site_kind(lbm_ctx* c, int8_t* kind) {
  if (!c || !kind) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  const int orc = refresh_owner_map(c);
  if (orc != LBM_OK) return orc;
  std::vector<int> m(c->NT);
  HIP_TRY(hipMemcpyAsync(m.data(), c->own, sizeof(int) * c->NT, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int64_t s = 0; s < c->NT; s++) kind[s] = m[s] == kEmpty ? 0 : (int8_t)(1 + (m[s] & 1));
  return check_status(c);
}

int lbm_shifts(lbm_ctx* c, int32_t* k) {
  if (!c || !k) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  if (c->np > 0) HIP_TRY(hipMemcpyAsync(k, c->P.k, sizeof(int) * 3 * c->np, hipMemcpyDeviceToHost, c->stream));
  return check_status(c);
}

int lbm_particle_info(lbm_ctx* c, int32_t p, int32_t* nbs, int32_t* nis) {
  if (!c || p < 0 || p >= c->np) return LBM_EINVAL;
  if (nbs) *nbs = c->h_nbs[p];
  if (nis) *nis = c->h_nis[p];
  return LBM_OK;
}

int lbm_get_distributions(lbm_ctx* c, double* f) {
  if (!c || !f) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  const int64_t n = (int64_t)c->q * c->PS;  // the device array (whole blocks)
  const int ss = (int)store_size(c->prm.storage);
  std::vector<unsigned char> h((size_t)n * ss);
  if (c->prm.aa) {
    // one array: gather the post-propagation values on the host
    HIP_TRY(hipMemcpyAsync(h.data(), c->f[0], (size_t)n * ss, hipMemcpyDeviceToHost, c->stream));
  } else {
    void* stage = c->f[1 - c->cur];
    const int rc = DISPATCH(c, launch_shift, c, c->f[c->cur], stage, 1);
    if (rc != LBM_OK) return rc;
    HIP_TRY(hipMemcpyAsync(h.data(), stage, (size_t)n * ss, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  // element of the host copy that holds f_i of site s
  const int lay = state_layout(c);
  std::vector<int64_t> src;
  if (lay == kLayAASwap) {
    src.resize((size_t)c->q * c->NT);
    for (const Geo& g : c->boxes)
      for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
          for (int x = 0; x < g.nx; x++)
            for (int i = 0; i < c->q; i++) {
              const int cx = c->q == 9 ? Lattice<9>::cx(i) : Lattice<19>::cx(i);
              const int cy = c->q == 9 ? Lattice<9>::cy(i) : Lattice<19>::cy(i);
              const int cz = c->q == 9 ? Lattice<9>::cz(i) : Lattice<19>::cz(i);
              const int o = c->q == 9 ? opposite<9>(i) : opposite<19>(i);
              const int64_t from = g.off + wrap(x - cx, g.nx) + (int64_t)g.nx * (wrap(y - cy, g.ny) +
                                                                                  (int64_t)g.ny * wrap(z - cz, g.nz));
              src[(size_t)i * c->NT + g.off + x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] = pop_elem(c->q, o, from);
            }
  }
  for (int i = 0; i < c->q; i++) {
    const double w = lattice_w(c->q, i);
    const double base = w * c->prm.rho0;
    for (int64_t s = 0; s < c->NT; s++) {
      const int64_t k = src.empty() ? pop_elem(c->q, i, s) : src[(size_t)i * c->NT + s];
      double g;
      switch (c->prm.storage) {
        case LBM_FP64: g = ((const double*)h.data())[k]; break;
        case LBM_FP32: g = ((const float*)h.data())[k]; break;
        case LBM_FP16: g = (double)(float)((const _Float16*)h.data())[k] * pop_unit<_Float16>(w); break;
        default: g = (double)bf16_bits_to_f32(((const uint16_t*)h.data())[k]) * pop_unit<bf16s>(w); break;
      }
      f[(int64_t)i * c->NT + s] = base + g;
    }
  }
  return check_status(c);
}

int lbm_set_distributions(lbm_ctx* c, const double* f) {
  if (!c || !f) return LBM_EINVAL;
  if (c->failed) return LBM_EHIP;
  const int64_t nf = (int64_t)c->q * c->NT;
  for (int64_t i = 0; i < nf; i++)
    if (!std::isfinite(f[i])) return LBM_ENONFINITE;
  void* stage = c->f[1 - c->cur];
  const int64_t n = (int64_t)c->q * c->PS;  // the device array (whole blocks; the tail zero)
  const int ss = (int)store_size(c->prm.storage);
  std::vector<unsigned char> h((size_t)n * ss, 0);
  for (int i = 0; i < c->q; i++) {
    const double w = lattice_w(c->q, i);
    const double base = w * c->prm.rho0;
    for (int64_t s = 0; s < c->NT; s++) {
      const int64_t k = pop_elem(c->q, i, s);
      const double g = f[(int64_t)i * c->NT + s] - base;
      switch (c->prm.storage) {
        case LBM_FP64: ((double*)h.data())[k] = g; break;
        case LBM_FP32: ((float*)h.data())[k] = (float)g; break;
        case LBM_FP16: ((_Float16*)h.data())[k] = (_Float16)(g / pop_unit<_Float16>(w)); break;
        default: ((uint16_t*)h.data())[k] = f32_to_bf16_bits((float)(g / pop_unit<bf16s>(w))); break;
      }
    }
  }
  if (c->prm.aa) {
    // the given populations are the complete post-propagation state: the
    // AA pattern's post-propagation half (the next step is an even one)
    HIP_TRY(hipMemcpyAsync(c->f[0], h.data(), (size_t)n * ss, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->cur = 0;
    return LBM_OK;
  }
  HIP_TRY(hipMemcpyAsync(stage, h.data(), (size_t)n * ss, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  // the given populations are the complete post-propagation state
  const int rc = DISPATCH(c, launch_shift, c, stage, c->f[c->cur], -1);
  if (rc != LBM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_set_profiling(lbm_ctx* c, int32_t on) {
  if (!c) return LBM_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->prof = on != 0;
  c->ev_used = 0;
  return LBM_OK;
}

int lbm_profile(lbm_ctx* c, double* sweep_ms, int64_t* sweeps) {
  if (!c) return LBM_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  double tot = 0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    tot += ms;
  }
  if (sweep_ms) *sweep_ms = tot;
  if (sweeps) *sweeps = (int64_t)(c->ev_used / 2);
  c->ev_used = 0;
  return LBM_OK;
}

int lbm_device_copy(void* dst, const void* src, size_t bytes, int32_t streaming_loads, void* hip_stream) {
  if (!dst || !src || bytes % 16 || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16)) return LBM_EINVAL;
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return LBM_OK;
  if (blocks_for(n) > 0x7fffffff) return LBM_EINVAL;
  if (streaming_loads)
    k_copy16<true><<<blocks_for(n), 256, 0, (hipStream_t)hip_stream>>>((const v4u*)src, (v4u*)dst, n);
  else
    k_copy16<false><<<blocks_for(n), 256, 0, (hipStream_t)hip_stream>>>((const v4u*)src, (v4u*)dst, n);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EWORKSPACE: return "workspace missing, misaligned or too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EOVERLAP: return "particles overlap";
    case LBM_ECAPACITY: return "capacity exceeded";
    case LBM_ENONFINITE: return "non-finite value";
    case LBM_EUNSUPPORTED: return "storage mode not supported";
    case LBM_ECOLLISION: return "collision search bound exceeded";
    case LBM_ESTATE: return "inconsistent device state: a boundary-site record named no entry";
    default: return "unknown error";
  }
}

}  // extern "C"
