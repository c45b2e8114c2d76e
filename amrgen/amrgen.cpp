// amrgen — seeded synthetic AMR octree scenes.
//
// This module only produces INPUTS: a list of octree leaves (level, integer
// cell coordinates) and the fp32 fields they carry.  It contains none of the
// renderer's arithmetic (no restriction, no rays, no traversal); both the CPU
// oracle and the GPU library consume its output as plain data.
//
// Scenes (box = [0,1)^3, root = level 0, a level-l cell has side 2^-l):
//   * BLOBS: 8 isotropic Gaussian blobs on a 1e-3 floor, times per-cell
//     lognormal noise exp(0.5 z - 0.125); a cell is refined while its noisy
//     density exceeds a threshold tau.
//   * DISK:  exponential galaxy disk rho0 exp(-R/3 kpc - |z|/0.3 kpc) in a
//     50 kpc box, times a unit-variance lognormal clump field exp(g - 1/2)
//     (g = sum of 64 random cosine modes, wavelengths log-uniform in
//     [0.1, 3] kpc), a 1e-6 floor and, optionally, 16 point-like "cores"
//     rho_k(r) = kappa^3 m_thr / max(r, r_min)^3 that force refinement down to
//     the deepest level.  A cell is refined while rho * dx^3 > m_thr.
//     Velocity: circular rotation v_c(R) = 220 R / sqrt(R^2 + 1 kpc^2) km/s
//     plus 10 km/s isotropic Gaussian dispersion, drawn per leaf.
//
// Randomness: SplitMix64.  Scene-level parameters come from a SplitMix64
// stream seeded by the scene seed; per-cell draws use a counter-based key
// (seed, stream, level, ix, iy, iz) hashed through the SplitMix64 output
// mixer, so every cell's draw is independent of traversal order and thread
// count.  Leaves are emitted depth-first in Morton child order (bit0 = x,
// bit1 = y, bit2 = z) below each base cell, base cells in Morton order.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

extern "C" {

typedef struct {
  int32_t kind;           // 0 = BLOBS, 1 = DISK
  int32_t levelmin;       // every cell above this level is refined
  int32_t lmax;           // no cell is refined at this level
  int32_t with_cores;     // DISK: add the point-like cores
  int32_t with_velocity;  // DISK: emit 3 velocity fields after density
  int32_t ncores;         // DISK: number of cores (16)
  int32_t nmodes;         // DISK: number of cosine modes (64)
  int32_t pad_;
  uint64_t seed;
  double threshold;       // BLOBS: tau; DISK: m_thr in rho0 * kpc^3
  double kappa;           // DISK: core strength (4)
} amrgen_params;

typedef struct {
  int64_t n;              // number of leaves
  int32_t nfields;        // 1 (density) or 4 (density, vx, vy, vz)
  int32_t lmax_reached;   // deepest leaf level
  int32_t* level;
  int32_t* ix;
  int32_t* iy;
  int32_t* iz;
  float* fields;          // [nfields][n]
} amrgen_leaves;

}  // extern "C"

namespace {

constexpr uint64_t kGold = 0x9e3779b97f4a7c15ULL;
constexpr double kPi = 3.14159265358979323846;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

struct SplitMix64 {
  uint64_t s;
  uint64_t next() { s += kGold; return mix64(s); }
  double u01() { return (static_cast<double>(next() >> 11) + 0.5) * 0x1.0p-53; }
  double uniform(double a, double b) { return a + (b - a) * u01(); }
};

inline uint64_t cell_key(uint64_t seed, uint64_t stream, int level, uint32_t ix,
                         uint32_t iy, uint32_t iz) {
  uint64_t h = mix64(seed * kGold + stream);
  h = mix64(h + kGold + static_cast<uint64_t>(level));
  h = mix64(h + kGold + ix);
  h = mix64(h + kGold + iy);
  h = mix64(h + kGold + iz);
  return h;
}
inline double u01_of(uint64_t h) { return (static_cast<double>(h >> 11) + 0.5) * 0x1.0p-53; }

// Standard normal for a cell by Box-Muller from two counter draws.
inline double cell_normal(uint64_t seed, uint64_t stream, int level, uint32_t ix, uint32_t iy,
                          uint32_t iz) {
  double u1 = u01_of(cell_key(seed, 2 * stream, level, ix, iy, iz));
  double u2 = u01_of(cell_key(seed, 2 * stream + 1, level, ix, iy, iz));
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * kPi * u2);
}

struct Blob { double c[3], inv2s2; };
struct Mode { double k[3], phase; };
struct Core { double x[3]; };

struct Scene {
  amrgen_params p;
  std::vector<Blob> blobs;
  std::vector<Mode> modes;
  std::vector<Core> cores;
  double box_kpc = 50.0;
  double rmin = 0.0;      // core softening, kpc
  double core_amp = 0.0;  // kappa^3 m_thr
  double gnorm = 0.0;     // sqrt(2 / nmodes)

  void init(const amrgen_params& prm) {
    p = prm;
    SplitMix64 rng{p.seed * 0xd1b54a32d192ed03ULL + 0x1234567ULL};
    if (p.kind == 0) {
      for (int k = 0; k < 8; ++k) {
        Blob b;
        for (int a = 0; a < 3; ++a) b.c[a] = rng.uniform(0.15, 0.85);
        double s = rng.uniform(0.02, 0.1);
        b.inv2s2 = 1.0 / (2.0 * s * s);
        blobs.push_back(b);
      }
    } else {
      for (int m = 0; m < p.nmodes; ++m) {
        double ct = 2.0 * rng.u01() - 1.0;
        double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        double ph = 2.0 * kPi * rng.u01();
        double lam = std::exp(rng.uniform(std::log(0.1), std::log(3.0)));
        double kk = 2.0 * kPi / lam;
        Mode md;
        md.k[0] = kk * st * std::cos(ph);
        md.k[1] = kk * st * std::sin(ph);
        md.k[2] = kk * ct;
        md.phase = 2.0 * kPi * rng.u01();
        modes.push_back(md);
      }
      gnorm = std::sqrt(2.0 / p.nmodes);
      for (int k = 0; k < p.ncores; ++k) {
        double R = rng.uniform(0.5, 8.0);
        double ph = 2.0 * kPi * rng.u01();
        double z = rng.uniform(-0.1, 0.1);
        Core c;
        c.x[0] = R * std::cos(ph);
        c.x[1] = R * std::sin(ph);
        c.x[2] = z;
        cores.push_back(c);
      }
      rmin = box_kpc * std::ldexp(1.0, -p.lmax);
      core_amp = p.kappa * p.kappa * p.kappa * p.threshold;
    }
  }

  // Physical position (kpc, centred) of a cell centre.
  void centre_kpc(int level, uint32_t ix, uint32_t iy, uint32_t iz, double x[3]) const {
    double h = std::ldexp(1.0, -level);
    x[0] = ((ix + 0.5) * h - 0.5) * box_kpc;
    x[1] = ((iy + 0.5) * h - 0.5) * box_kpc;
    x[2] = ((iz + 0.5) * h - 0.5) * box_kpc;
  }

  double disk_density(const double x[3]) const {
    double R = std::sqrt(x[0] * x[0] + x[1] * x[1]);
    double g = 0.0;
    for (const Mode& m : modes)
      g += std::cos(m.k[0] * x[0] + m.k[1] * x[1] + m.k[2] * x[2] + m.phase);
    g *= gnorm;
    double rho = 1e-6 + std::exp(-R / 3.0 - std::fabs(x[2]) / 0.3) * std::exp(g - 0.5);
    if (p.with_cores) {
      for (const Core& c : cores) {
        double dx = x[0] - c.x[0], dy = x[1] - c.x[1], dz = x[2] - c.x[2];
        double r = std::max(std::sqrt(dx * dx + dy * dy + dz * dz), rmin);
        rho += core_amp / (r * r * r);
      }
    }
    return rho;
  }

  double blob_density(int level, uint32_t ix, uint32_t iy, uint32_t iz) const {
    double h = std::ldexp(1.0, -level);
    double x = (ix + 0.5) * h, y = (iy + 0.5) * h, z = (iz + 0.5) * h;
    double rho = 1e-3;
    for (const Blob& b : blobs) {
      double dx = x - b.c[0], dy = y - b.c[1], dz = z - b.c[2];
      rho += std::exp(-(dx * dx + dy * dy + dz * dz) * b.inv2s2);
    }
    double noise = std::exp(0.5 * cell_normal(p.seed, 1, level, ix, iy, iz) - 0.125);
    return rho * noise;
  }
};

struct LeafRec {
  uint32_t ix, iy, iz;
  uint8_t level;
  float f[4];
};

struct Chunk {
  std::vector<LeafRec> recs;
  int64_t count = 0;
  int lmax = 0;
};

void refine(const Scene& sc, int level, uint32_t ix, uint32_t iy, uint32_t iz, bool count_only,
            Chunk& out) {
  const amrgen_params& p = sc.p;
  double rho;
  double xk[3];
  bool split;
  if (p.kind == 0) {
    rho = sc.blob_density(level, ix, iy, iz);
    split = level < p.lmax && rho > p.threshold;
  } else {
    sc.centre_kpc(level, ix, iy, iz, xk);
    rho = sc.disk_density(xk);
    double dx = sc.box_kpc * std::ldexp(1.0, -level);
    split = level < p.lmax && rho * dx * dx * dx > p.threshold;
  }
  if (level < p.levelmin) split = true;
  if (split) {
    for (int c = 0; c < 8; ++c)
      refine(sc, level + 1, 2 * ix + (c & 1), 2 * iy + ((c >> 1) & 1), 2 * iz + ((c >> 2) & 1),
             count_only, out);
    return;
  }
  out.count++;
  out.lmax = std::max(out.lmax, level);
  if (count_only) return;
  LeafRec r;
  r.ix = ix; r.iy = iy; r.iz = iz; r.level = static_cast<uint8_t>(level);
  r.f[0] = static_cast<float>(rho);
  r.f[1] = r.f[2] = r.f[3] = 0.0f;
  if (p.kind == 1 && p.with_velocity) {
    double R = std::sqrt(xk[0] * xk[0] + xk[1] * xk[1]);
    double vc = 220.0 * R / std::sqrt(R * R + 1.0);
    double ex = 0.0, ey = 0.0;
    if (R > 0.0) { ex = -xk[1] / R; ey = xk[0] / R; }
    double zx = cell_normal(p.seed, 11, level, ix, iy, iz);
    double zy = cell_normal(p.seed, 12, level, ix, iy, iz);
    double zz = cell_normal(p.seed, 13, level, ix, iy, iz);
    r.f[1] = static_cast<float>(vc * ex + 10.0 * zx);
    r.f[2] = static_cast<float>(vc * ey + 10.0 * zy);
    r.f[3] = static_cast<float>(10.0 * zz);
  }
  out.recs.push_back(r);
}

inline uint32_t compact1by2(uint64_t x) {
  uint32_t r = 0;
  for (int b = 0; b < 21; ++b) r |= static_cast<uint32_t>((x >> (3 * b)) & 1u) << b;
  return r;
}

}  // namespace

extern "C" {

void amrgen_free(amrgen_leaves* L) {
  if (!L) return;
  std::free(L->level); std::free(L->ix); std::free(L->iy); std::free(L->iz);
  std::free(L->fields);
  std::memset(L, 0, sizeof(*L));
}

// Generate a scene.  count_only != 0 fills only n and lmax_reached.
// Returns 0 on success, -1 on bad parameters, -2 on allocation failure.
int amrgen_generate(const amrgen_params* prm, amrgen_leaves* out, int count_only, int nthreads) {
  if (!prm || !out) return -1;
  if (prm->kind < 0 || prm->kind > 1) return -1;
  if (prm->levelmin < 0 || prm->levelmin > 9 || prm->lmax < prm->levelmin || prm->lmax > 24)
    return -1;
  std::memset(out, 0, sizeof(*out));
  Scene sc;
  sc.init(*prm);
  const int64_t nbase = int64_t(1) << (3 * prm->levelmin);
  const int64_t nchunks = std::min<int64_t>(nbase, 4096);
  std::vector<Chunk> chunks(nchunks);
  std::atomic<int64_t> next{0};
  if (nthreads <= 0) nthreads = static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
  auto worker = [&]() {
    for (;;) {
      int64_t c = next.fetch_add(1);
      if (c >= nchunks) break;
      int64_t b0 = nbase * c / nchunks, b1 = nbase * (c + 1) / nchunks;
      for (int64_t b = b0; b < b1; ++b) {
        uint64_t m = static_cast<uint64_t>(b);
        refine(sc, prm->levelmin, compact1by2(m), compact1by2(m >> 1), compact1by2(m >> 2),
               count_only != 0, chunks[c]);
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) th.emplace_back(worker);
  for (auto& t : th) t.join();

  int64_t n = 0;
  int lmax = 0;
  for (auto& ch : chunks) { n += ch.count; lmax = std::max(lmax, ch.lmax); }
  out->n = n;
  out->lmax_reached = lmax;
  out->nfields = (prm->kind == 1 && prm->with_velocity) ? 4 : 1;
  if (count_only) return 0;
  const int nf = out->nfields;
  out->level = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * std::max<int64_t>(n, 1)));
  out->ix = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * std::max<int64_t>(n, 1)));
  out->iy = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * std::max<int64_t>(n, 1)));
  out->iz = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * std::max<int64_t>(n, 1)));
  out->fields = static_cast<float*>(std::malloc(sizeof(float) * nf * std::max<int64_t>(n, 1)));
  if (!out->level || !out->ix || !out->iy || !out->iz || !out->fields) {
    amrgen_free(out);
    return -2;
  }
  std::vector<int64_t> offs(nchunks + 1, 0);
  for (int64_t c = 0; c < nchunks; ++c) offs[c + 1] = offs[c] + chunks[c].count;
  next = 0;
  auto copier = [&]() {
    for (;;) {
      int64_t c = next.fetch_add(1);
      if (c >= nchunks) break;
      int64_t o = offs[c];
      for (const LeafRec& r : chunks[c].recs) {
        out->level[o] = r.level; out->ix[o] = r.ix; out->iy[o] = r.iy; out->iz[o] = r.iz;
        for (int f = 0; f < nf; ++f) out->fields[f * n + o] = r.f[f];
        ++o;
      }
      std::vector<LeafRec>().swap(chunks[c].recs);
    }
  };
  th.clear();
  for (int t = 0; t < nthreads; ++t) th.emplace_back(copier);
  for (auto& t : th) t.join();
  return 0;
}

// Scene-level core positions in box units (for aiming cameras at core k).
int amrgen_core_position(const amrgen_params* prm, int k, double* xyz_box) {
  if (!prm || prm->kind != 1 || k < 0 || k >= prm->ncores) return -1;
  Scene sc;
  sc.init(*prm);
  for (int a = 0; a < 3; ++a) xyz_box[a] = sc.cores[k].x[a] / sc.box_kpc + 0.5;
  return 0;
}

}  // extern "C"
