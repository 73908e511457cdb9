// TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT PATH.
//
// Plain, slow, FP64 CPU oracle for the moving-mesh finite-volume step of
// Chang, Wadsley & Quinn (2017), "A moving mesh hydrodynamic solver for
// ChaNGa" (MANGA).  It exists so that the HIP path can be checked against an
// independent, obviously-correct implementation.  Only the tests, the smoke
// check and the benchmark's CPU-baseline leg may load it; the library under
// paper_1707_05333_amd/ never links, includes or calls it, and the two share
// no code.
//
// Arithmetic is IEEE double throughout (compiled without fast-math).  Every
// function names the passage of the paper it follows.  Where the paper is
// silent or garbled, the reading taken is stated where it is used:
//   R-upd   update sign: F is the flux from i to j along the face normal;
//           Q_i loses dt*A*F, Q_j gains it (Sec. 4, update of the charges).
//   R-s10   S10 limiter displacement is c_j - c_i (+ periodic shift); the
//           extrema include cell i itself (Sec. 4.1, limiter definition).
//   R-dm    the Duffell-MacFadyen factor reads max[theta dU/Delta, 0]
//           clamped to 1, applied per face at reconstruction, with Delta the
//           gradient's extrapolation from the cell centroid to the face
//           centroid.  Then theta <= 1/2 is exactly the condition that the two
//           reconstructed face states never cross, which is the paper's TVD
//           statement for theta < 0.5 (Sec. 4.1).
//   R-grad  gradients are area-weighted least squares about the cell
//           centroids (the paper cites a centroid-based estimate whose
//           formula it does not print, Sec. 4.1).
//   R-pred  the half-step rate follows the moving generator:
//           dU/dt = -div F + w . grad U (Sec. 4.1, eqs. for the time
//           derivative and the half-step state; Sec. 4 item 2).
//   R-hllc  HLLC with Davis wave-speed bounds, written in normal/tangential
//           form (Sec. 4 items 3-5; the paper follows Toro 2009).  The HLL
//           alternative (same item) uses the same wave-speed bounds.
//   R-floor floors keep the velocity and pressure and raise the density, or
//           keep density and velocity and raise the pressure (Sec. 4.1,
//           floors paragraph; values are not given by the paper).  A face
//           state whose reconstruction would need a floor is replaced by its
//           cell's half-step state (first order on that side of the face):
//           component-wise extrapolation across a large density jump can
//           pair a small density with a large momentum, a velocity that no
//           floor repairs.
//   R-box   the starting cell is the box r_i +- L/2, the exact Voronoi cell
//           of i's own periodic images (Sec. 3, the large box each cell is cut from).
//   R-area  a face is kept iff its computed area is positive.  (A threshold
//           relative to each cell's own volume would differ between the two
//           cells of a face and keep a face on one side only.)
//   R-dt    dt = min(dt_max, min_i dt_i); no power-of-two rungs (Sec. 4.2).
//   R-w     the mesh velocity of a step is evaluated from the state at the
//           start of the step and used both for the face velocities and
//           the drift (Sec. 2 outline; Sec. 4.2).
//   R-ent   entropy switch (Sec. 4.3): the state gains X = rho A with the
//           entropic function A = P rho^-gamma, advected by the mass flux
//           (its face value upwind by the contact, A_K = X_K / rho_K from
//           the reconstructed, pre-floor face state).  The shock Mach number
//           of a face is sqrt(1 + (gamma+1)/(2 gamma) max(0, p*/P_K - 1))
//           maximised over its two sides, with p* the HLLC star pressure;
//           a cell's Mach number is the maximum over its faces.  Cells below
//           the threshold take the pressure from the entropy, the others keep
//           the energy and reset X from the new state.
//   R-tess  optional half-step geometry (Sec. 6, first future improvement:
//           rebuild the tessellation at the half step): the predictor runs
//           on the time-n mesh; the generators are moved by w dt/2, the
//           mesh is rebuilt there, and the second gradient, the face
//           states and the fluxes use that mesh; the floors after the
//           update use its volumes; the drift is still r^n + w dt.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm2(V3 a) { return dot(a, a); }
inline double comp(V3 a, int c) { return c == 0 ? a.x : (c == 1 ? a.y : a.z); }

// Periodic image code: k in {-1,0,1}^3  ->  (kx+1) + 3(ky+1) + 9(kz+1).
inline int kcode(int kx, int ky, int kz) { return (kx + 1) + 3 * (ky + 1) + 9 * (kz + 1); }
inline void kdecode(int code, int k[3]) {
  k[0] = code % 3 - 1;
  k[1] = (code / 3) % 3 - 1;
  k[2] = code / 9 - 1;
}
inline int kneg(int code) { return 26 - code; }

constexpr double kPi = 3.14159265358979323846;

// ===========================================================================
// O1: the Voronoi cell of one generator by half-space clipping (Sec. 3).
// Coordinates are relative to the generator r_i, so the bisector of r_i and a
// neighbour image at relative position d is {x : d.x <= |d|^2/2}.
// ===========================================================================

struct Plane {
  int j;      // neighbour index (== i for the generator's own images)
  int code;   // periodic image code of the neighbour
  V3 d;       // neighbour image position relative to r_i
  double h;   // |d|^2 / 2
};

struct Face {
  int plane;            // index into Poly::planes
  std::vector<V3> v;    // polygon, counter-clockwise seen from outside
};

struct Poly {
  std::vector<Plane> planes;
  std::vector<Face> faces;
};

// Signed area vector of a polygon by a fan from its first vertex.
V3 area_vector(const std::vector<V3>& v) {
  V3 s{0, 0, 0};
  for (size_t k = 1; k + 1 < v.size(); ++k) s = s + 0.5 * cross(v[k] - v[0], v[k + 1] - v[0]);
  return s;
}

// R-box: the starting cell is the box r_i +- L/2, bounded by the bisectors
// of r_i and its six axis images.
void init_box(Poly& P, int i, V3 L) {
  P.planes.clear();
  P.faces.clear();
  const double Lc[3] = {L.x, L.y, L.z};
  for (int a = 0; a < 3; ++a) {
    for (int s = 1; s >= -1; s -= 2) {
      int k[3] = {0, 0, 0};
      k[a] = s;
      Plane pl;
      pl.j = i;
      pl.code = kcode(k[0], k[1], k[2]);
      pl.d = {k[0] * Lc[0], k[1] * Lc[1], k[2] * Lc[2]};
      pl.h = 0.5 * norm2(pl.d);
      P.planes.push_back(pl);
    }
  }
  const double hx = 0.5 * L.x, hy = 0.5 * L.y, hz = 0.5 * L.z;
  for (int p = 0; p < 6; ++p) {
    const int a = p / 2;
    const double s = (p % 2 == 0) ? 1.0 : -1.0;
    // Four corners of the face; the two free axes are the other two.
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double half[3] = {hx, hy, hz};
    std::vector<V3> v;
    const double sb[4] = {-1, 1, 1, -1}, sc[4] = {-1, -1, 1, 1};
    for (int q = 0; q < 4; ++q) {
      double x[3];
      x[a] = s * half[a];
      x[b] = sb[q] * half[b];
      x[c] = sc[q] * half[c];
      v.push_back({x[0], x[1], x[2]});
    }
    // Orient counter-clockwise seen from outside (area vector along d).
    if (dot(area_vector(v), P.planes[p].d) < 0) std::reverse(v.begin(), v.end());
    P.faces.push_back({p, v});
  }
}

// Point where the polyhedron edge from an inside vertex to an outside vertex
// crosses the plane.  Always evaluated with the inside vertex first, so the
// two faces sharing the edge produce the identical point.
V3 cross_point(const Plane& pl, V3 in, V3 out) {
  const double din = dot(pl.d, in), dout = dot(pl.d, out);
  const double t = (pl.h - din) / (dout - din);
  return in + t * (out - in);
}

double max_vertex_r2(const Poly& P) {
  double r2 = 0;
  for (const Face& F : P.faces)
    for (const V3& v : F.v) r2 = std::max(r2, norm2(v));
  return r2;
}

// Cut the cell by the bisector plane of one neighbour image (Sec. 3: the
// plane that bisects the segment to the neighbour).  A vertex is outside iff
// d.v > |d|^2/2 in plain FP64.  Returns true if the cell changed.
bool clip(Poly& P, const Plane& pl) {
  bool any_out = false;
  for (const Face& F : P.faces) {
    for (const V3& v : F.v)
      if (dot(pl.d, v) > pl.h) { any_out = true; break; }
    if (any_out) break;
  }
  if (!any_out) return false;

  const int new_plane = (int)P.planes.size();
  std::vector<Face> kept;
  std::vector<V3> exits;
  for (const Face& F : P.faces) {
    const size_t n = F.v.size();
    std::vector<char> out(n);
    size_t nout = 0;
    for (size_t k = 0; k < n; ++k) {
      out[k] = dot(pl.d, F.v[k]) > pl.h;
      nout += out[k];
    }
    if (nout == n) continue;        // face entirely cut away
    if (nout == 0) { kept.push_back(F); continue; }
    Face G{F.plane, {}};
    for (size_t k = 0; k < n; ++k) {
      const V3 a = F.v[k], b = F.v[(k + 1) % n];
      const bool ia = !out[k], ib = !out[(k + 1) % n];
      if (ia) G.v.push_back(a);
      if (ia && !ib) {
        const V3 X = cross_point(pl, a, b);
        G.v.push_back(X);
        exits.push_back(X);   // each crossing edge is an exit in exactly one face
      } else if (!ia && ib) {
        G.v.push_back(cross_point(pl, b, a));
      }
    }
    kept.push_back(G);
  }
  // The new face: the crossing points ordered by angle about the plane
  // normal (counter-clockwise seen from outside).
  if (exits.size() >= 3) {
    V3 m{0, 0, 0};
    for (const V3& X : exits) m = m + X;
    m = (1.0 / exits.size()) * m;
    const V3 nhat = (1.0 / std::sqrt(norm2(pl.d))) * pl.d;
    V3 e1 = exits[0] - m;
    e1 = e1 - dot(e1, nhat) * nhat;
    e1 = (1.0 / std::sqrt(norm2(e1))) * e1;
    const V3 e2 = cross(nhat, e1);
    std::vector<std::pair<double, V3>> ang;
    for (const V3& X : exits) ang.push_back({std::atan2(dot(X - m, e2), dot(X - m, e1)), X});
    std::sort(ang.begin(), ang.end(), [](const std::pair<double, V3>& a, const std::pair<double, V3>& b) {
      return a.first < b.first;
    });
    Face N{new_plane, {}};
    for (auto& pr : ang) N.v.push_back(pr.second);
    kept.push_back(N);
  }
  P.planes.push_back(pl);
  P.faces.swap(kept);
  return true;
}

// Geometry of a finished cell (Sec. 4: charges need V_i; Sec. 4.1: centre of
// mass c_i; face areas A_ij and face centres for the fluxes).
struct CellOut {
  double V = 0;       // volume
  V3 c_rel{0, 0, 0};  // centroid minus generator
  double vtet = 0;    // volume by an independent tetrahedral decomposition
  double rmax = 0;    // farthest vertex distance
  int nvert = 0;      // number of distinct vertices
  std::vector<int> j, code;
  std::vector<double> A;
  std::vector<V3> f_rel;  // face area centroid minus generator
  double delta = 1e300;   // non-degeneracy margin (see certificate())
  int status = 0;
};

void finish_cell(const Poly& P, CellOut& out) {
  struct FG { int plane; double A; V3 f; double dist; };
  std::vector<FG> fg;
  double V = 0;
  V3 mom{0, 0, 0};
  for (const Face& F : P.faces) {
    const Plane& pl = P.planes[F.plane];
    const V3 nhat = (1.0 / std::sqrt(norm2(pl.d))) * pl.d;
    double A = 0;
    V3 S{0, 0, 0};
    for (size_t k = 1; k + 1 < F.v.size(); ++k) {
      const double a = 0.5 * dot(cross(F.v[k] - F.v[0], F.v[k + 1] - F.v[0]), nhat);
      A += a;
      S = S + (a / 3.0) * (F.v[0] + F.v[k] + F.v[k + 1]);
    }
    if (!(A > 0)) continue;   // R-area: a plane that only touches the cell
    const V3 f = (1.0 / A) * S;
    const double dist = 0.5 * std::sqrt(norm2(pl.d));   // generator-to-face distance
    // Pyramid with apex at the generator: volume A*dist/3, centroid 3/4 of
    // the way from the apex to the base centroid.
    const double vol = A * dist / 3.0;
    V += vol;
    mom = mom + (0.75 * vol) * f;
    fg.push_back({F.plane, A, f, dist});
  }
  out.V = V;
  out.c_rel = (1.0 / V) * mom;
  // Independent volume: tetrahedra from one vertex of the cell.
  if (!P.faces.empty() && !P.faces[0].v.empty()) {
    const V3 apex = P.faces[0].v[0];
    double vt = 0;
    for (const Face& F : P.faces)
      for (size_t k = 1; k + 1 < F.v.size(); ++k)
        vt += dot(F.v[0] - apex, cross(F.v[k] - apex, F.v[k + 1] - apex)) / 6.0;
    out.vtet = vt;
  }
  out.rmax = std::sqrt(max_vertex_r2(P));
  // Distinct vertices via Euler's formula for a convex polyhedron.
  size_t half_edges = 0;
  for (const Face& F : P.faces) half_edges += F.v.size();
  out.nvert = (int)(2 + half_edges / 2 - P.faces.size());
  // Faces ordered by (j, image code).
  std::vector<size_t> idx;
  for (size_t q = 0; q < fg.size(); ++q) idx.push_back(q);
  std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    const Plane& pa = P.planes[fg[a].plane];
    const Plane& pb = P.planes[fg[b].plane];
    return std::make_pair(pa.j, pa.code) < std::make_pair(pb.j, pb.code);
  });
  for (size_t q : idx) {
    const Plane& pl = P.planes[fg[q].plane];
    out.j.push_back(pl.j);
    out.code.push_back(pl.code);
    out.A.push_back(fg[q].A);
    out.f_rel.push_back(fg[q].f);
  }
}

// Non-degeneracy certificate: the smallest margin (|v - q| - |v - r_i|)
// over the cell's vertices v and candidate images q that do not define v.
// Zero margin means five generators on one sphere, where the tessellation's
// topology is not stable under rounding.
double certificate(const Poly& P, const std::vector<Plane>& cands) {
  std::map<std::tuple<double, double, double>, std::set<std::pair<int, int>>> inc;
  for (const Face& F : P.faces) {
    const Plane& pl = P.planes[F.plane];
    for (const V3& v : F.v) inc[std::make_tuple(v.x, v.y, v.z)].insert({pl.j, pl.code});
  }
  double best = 1e300;
  for (auto& kv : inc) {
    const V3 v{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first)};
    const double rv = std::sqrt(norm2(v));
    for (const Plane& q : cands) {
      if (kv.second.count({q.j, q.code})) continue;
      best = std::min(best, std::sqrt(norm2(v - q.d)) - rv);
    }
  }
  return best;
}

struct Mesh {
  int64_t n = 0;
  V3 L{1, 1, 1};
  std::vector<V3> r;
  std::vector<CellOut> cells;
  double delta_min = 1e300;
  int status = 0;
};

Plane make_plane(const Mesh& M, int i, int j, int kx, int ky, int kz) {
  Plane pl;
  pl.j = j;
  pl.code = kcode(kx, ky, kz);
  const V3 s{kx * M.L.x, ky * M.L.y, kz * M.L.z};
  // The generator's own images are exactly k*L away.
  pl.d = (j == i) ? s : (M.r[j] + s) - M.r[i];
  pl.h = 0.5 * norm2(pl.d);
  return pl;
}

// Brute force: clip by every generator in every neighbouring periodic image.
// Unless `exhaustive`, a plane farther than the farthest vertex is skipped;
// that test is exact (such a plane cannot have a vertex strictly outside).
void build_cell_brute(const Mesh& M, int i, bool exhaustive, CellOut& out) {
  Poly P;
  init_box(P, i, M.L);
  double r2 = max_vertex_r2(P);
  for (int j = 0; j < M.n; ++j)
    for (int kz = -1; kz <= 1; ++kz)
      for (int ky = -1; ky <= 1; ++ky)
        for (int kx = -1; kx <= 1; ++kx) {
          if (j == i && kx == 0 && ky == 0 && kz == 0) continue;
          const Plane pl = make_plane(M, i, j, kx, ky, kz);
          if (!exhaustive && norm2(pl.d) >= 4.0 * r2) continue;
          if (clip(P, pl)) r2 = max_vertex_r2(P);
        }
  finish_cell(P, out);
  // Index-order clipping passes through near-degenerate intermediate cells,
  // where one vertex can be represented with last-bit differences in its
  // faces; the margin is therefore only computed on the distance-ordered
  // grid path.  Brute force reports NaN.
  out.delta = std::nan("");
}

// Grid path (Sec. 3): candidates from a periodic bucket grid, ordered by
// distance (ties by index, then image code); clipping stops at the first
// candidate farther than twice the farthest vertex.  The stencil grows by
// one ring whenever twice the farthest vertex exceeds the distance the
// current stencil is known to cover.
struct Grid {
  int nb[3];
  double hb[3];
  std::vector<int> start;   // bucket -> first slot in `order`
  std::vector<int> order;   // generators sorted by bucket, then index
};

int bucket_coord(double x, double h, int nb) {
  int b = (int)std::floor(x / h);
  if (b < 0) b = 0;
  if (b >= nb) b = nb - 1;
  return b;
}

Grid make_grid(const Mesh& M, double per_bucket) {
  Grid G;
  const double vol = M.L.x * M.L.y * M.L.z;
  const double hb = std::cbrt(vol / (double)M.n * per_bucket);
  const double Lc[3] = {M.L.x, M.L.y, M.L.z};
  for (int a = 0; a < 3; ++a) {
    G.nb[a] = std::max(1, (int)std::floor(Lc[a] / hb));
    G.hb[a] = Lc[a] / G.nb[a];
  }
  const int64_t nbt = (int64_t)G.nb[0] * G.nb[1] * G.nb[2];
  std::vector<int> key(M.n);
  std::vector<int> count(nbt + 1, 0);
  for (int64_t i = 0; i < M.n; ++i) {
    const int bx = bucket_coord(M.r[i].x, G.hb[0], G.nb[0]);
    const int by = bucket_coord(M.r[i].y, G.hb[1], G.nb[1]);
    const int bz = bucket_coord(M.r[i].z, G.hb[2], G.nb[2]);
    key[i] = bx + G.nb[0] * (by + G.nb[1] * bz);
    count[key[i] + 1]++;
  }
  for (int64_t b = 0; b < nbt; ++b) count[b + 1] += count[b];
  G.start = count;
  G.order.resize(M.n);
  std::vector<int> cur(count.begin(), count.end() - 1);
  for (int64_t i = 0; i < M.n; ++i) G.order[cur[key[i]]++] = (int)i;
  return G;
}

void build_cell_grid(const Mesh& M, const Grid& G, int i, CellOut& out, bool want_cert) {
  const V3 ri = M.r[i];
  const double x[3] = {ri.x, ri.y, ri.z};
  int b[3];
  for (int a = 0; a < 3; ++a) b[a] = bucket_coord(x[a], G.hb[a], G.nb[a]);
  for (int ring = 1;; ++ring) {
    if (ring > G.nb[0] || ring > G.nb[1] || ring > G.nb[2]) {
      build_cell_brute(M, i, false, out);
      return;
    }
    std::vector<Plane> cand;
    for (int oz = -ring; oz <= ring; ++oz)
      for (int oy = -ring; oy <= ring; ++oy)
        for (int ox = -ring; ox <= ring; ++ox) {
          const int o[3] = {ox, oy, oz};
          int bb[3], k[3];
          for (int a = 0; a < 3; ++a) {
            const int t = b[a] + o[a];
            k[a] = (t < 0) ? -1 : (t >= G.nb[a] ? 1 : 0);
            bb[a] = t - k[a] * G.nb[a];
          }
          const int key = bb[0] + G.nb[0] * (bb[1] + G.nb[1] * bb[2]);
          for (int s = G.start[key]; s < G.start[key + 1]; ++s) {
            const int j = G.order[s];
            if (j == i && k[0] == 0 && k[1] == 0 && k[2] == 0) continue;
            cand.push_back(make_plane(M, i, j, k[0], k[1], k[2]));
          }
        }
    std::sort(cand.begin(), cand.end(), [](const Plane& a, const Plane& c) {
      const double da = norm2(a.d), dc = norm2(c.d);
      if (da != dc) return da < dc;
      if (a.j != c.j) return a.j < c.j;
      return a.code < c.code;
    });
    Poly P;
    init_box(P, i, M.L);
    double r2 = max_vertex_r2(P);
    for (const Plane& pl : cand) {
      if (norm2(pl.d) >= 4.0 * r2) break;   // security radius (Sec. 3)
      if (clip(P, pl)) r2 = max_vertex_r2(P);
    }
    // Distance beyond which every generator image lies outside the stencil.
    double reach = 1e300;
    for (int a = 0; a < 3; ++a) {
      const double t = x[a] - b[a] * G.hb[a];
      reach = std::min(reach, ring * G.hb[a] + std::min(t, G.hb[a] - t));
    }
    if (4.0 * r2 <= reach * reach * (1.0 - 1e-12)) {
      finish_cell(P, out);
      if (want_cert) out.delta = certificate(P, cand);
      return;
    }
  }
}

// ===========================================================================
// Hydrodynamics on the tessellation (Sec. 4).
// ===========================================================================

struct Params {
  double box[3];
  double gamma, cfl, eta, chi, zeta, theta, rho_floor, p_floor;
  int32_t limiter_disp;     // 0: c_j - c_i (R-s10); 1: face centroid - c_i
  int32_t predictor_frame;  // 0: moving generator (R-pred); 1: Eulerian
  int32_t limit_mask;       // S10 limiter on: bit 0 time-n gradient, bit 1 half-step gradient (default 3)
  int32_t riemann;          // 0: HLLC (the paper's default), 1: HLL (Sec. 4 item 4)
  int32_t half_step_mesh;   // 1: fluxes on the mesh of the half-step positions (R-tess)
  int32_t pad;
  double mach_threshold;    // entropy switch (Sec. 4.3, R-ent): 0 = energy equation only
};

// R-floor (Sec. 4.1, floors paragraph).  U = (rho, m, E) densities.
// Returns the number of floors that fired (0, 1 or 2).
int apply_floors(double U[5], const Params& p) {
  const double g1 = p.gamma - 1.0;
  int hits = 0;
  double rho = U[0];
  if (rho < p.rho_floor) {
    double v[3] = {0, 0, 0};
    double P = p.p_floor;
    if (rho > 0) {
      for (int a = 0; a < 3; ++a) v[a] = U[1 + a] / rho;
      P = g1 * (U[4] - 0.5 * (U[1] * v[0] + U[2] * v[1] + U[3] * v[2]));
    }
    P = std::max(P, p.p_floor);
    rho = p.rho_floor;
    U[0] = rho;
    for (int a = 0; a < 3; ++a) U[1 + a] = rho * v[a];
    U[4] = P / g1 + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    hits++;
  }
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
  const double P = g1 * (U[4] - ke);
  if (P < p.p_floor) {
    U[4] = p.p_floor / g1 + ke;
    hits++;
  }
  return hits;
}

struct Prim {
  double rho, v[3], P;
};
Prim to_prim(const double U[5], double gamma) {
  Prim w;
  w.rho = U[0];
  for (int a = 0; a < 3; ++a) w.v[a] = U[1 + a] / U[0];
  w.P = (gamma - 1.0) * (U[4] - 0.5 * (U[1] * w.v[0] + U[2] * w.v[1] + U[3] * w.v[2]));
  return w;
}

V3 shift_of(const Mesh& M, int code) {
  int k[3];
  kdecode(code, k);
  return {k[0] * M.L.x, k[1] * M.L.y, k[2] * M.L.z};
}
V3 centroid(const Mesh& M, int i) { return M.r[i] + M.cells[i].c_rel; }

// Mesh velocity (Sec. 4.2): w = eta v + dw, with the roundness correction dw
// steering the generator toward the cell's centre of mass at chi c_s, ramped
// between 0.9 and 1.1 zeta R.  The per-cell CFL timestep uses the same R.
void mesh_velocity(const Mesh& M, const Params& p, int i, const double U[5], double w[3], double& dt_i) {
  const Prim pr = to_prim(U, p.gamma);
  const double cs = std::sqrt(p.gamma * pr.P / pr.rho);
  const double V = M.cells[i].V;
  const double R = std::cbrt(3.0 * V / (4.0 * kPi));
  const V3 d = M.cells[i].c_rel;   // c_i - r_i
  const double dn = std::sqrt(norm2(d));
  double ramp;
  if (dn < 0.9 * p.zeta * R) ramp = 0.0;
  else if (dn <= 1.1 * p.zeta * R) ramp = (dn - 0.9 * p.zeta * R) / (0.2 * p.zeta * R);
  else ramp = 1.0;
  double dw[3] = {0, 0, 0};
  if (dn > 0 && ramp > 0) {
    dw[0] = p.chi * cs * ramp * d.x / dn;
    dw[1] = p.chi * cs * ramp * d.y / dn;
    dw[2] = p.chi * cs * ramp * d.z / dn;
  }
  double rel2 = 0;
  for (int a = 0; a < 3; ++a) {
    w[a] = p.eta * pr.v[a] + dw[a];
    rel2 += (pr.v[a] - w[a]) * (pr.v[a] - w[a]);
  }
  dt_i = p.cfl * R / (cs + std::sqrt(rel2));
}

// R-grad + the S10 limiter (Sec. 4.1).  g_k = M^-1 sum_j w_ij (U_jk - U_ik) d_ij,
// d_ij = c_j + s - c_i, w_ij = A_ij / |d_ij|^2, M = sum_j w_ij d_ij d_ij^T.
void gradient_cell(const Mesh& M, const Params& p, int i, const double* U, double G[5][3], bool limit) {
  const CellOut& C = M.cells[i];
  const V3 ci = centroid(M, i);
  double Mm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double b[5][3] = {};
  std::vector<V3> dv(C.j.size());
  for (size_t e = 0; e < C.j.size(); ++e) {
    const int j = C.j[e];
    const V3 d = (centroid(M, j) + shift_of(M, C.code[e])) - ci;
    dv[e] = d;
    const double w = C.A[e] / norm2(d);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Mm[r][c] += w * comp(d, r) * comp(d, c);
    for (int q = 0; q < 5; ++q) {
      const double dU = U[5 * j + q] - U[5 * i + q];
      for (int r = 0; r < 3; ++r) b[q][r] += w * dU * comp(d, r);
    }
  }
  // Inverse of the symmetric 3x3 matrix by its adjugate.
  const double a00 = Mm[1][1] * Mm[2][2] - Mm[1][2] * Mm[2][1];
  const double a01 = Mm[0][2] * Mm[2][1] - Mm[0][1] * Mm[2][2];
  const double a02 = Mm[0][1] * Mm[1][2] - Mm[0][2] * Mm[1][1];
  const double a11 = Mm[0][0] * Mm[2][2] - Mm[0][2] * Mm[2][0];
  const double a12 = Mm[0][2] * Mm[1][0] - Mm[0][0] * Mm[1][2];
  const double a22 = Mm[0][0] * Mm[1][1] - Mm[0][1] * Mm[1][0];
  const double det = Mm[0][0] * a00 + Mm[0][1] * (Mm[1][2] * Mm[2][0] - Mm[1][0] * Mm[2][2]) +
                     Mm[0][2] * (Mm[1][0] * Mm[2][1] - Mm[1][1] * Mm[2][0]);
  const double inv[3][3] = {{a00 / det, a01 / det, a02 / det},
                            {a01 / det, a11 / det, a12 / det},
                            {a02 / det, a12 / det, a22 / det}};
  for (int q = 0; q < 5; ++q)
    for (int r = 0; r < 3; ++r) G[q][r] = inv[r][0] * b[q][0] + inv[r][1] * b[q][1] + inv[r][2] * b[q][2];
  if (!limit) return;
  for (int q = 0; q < 5; ++q) {
    const double Ui = U[5 * i + q];
    double umax = Ui, umin = Ui;
    for (size_t e = 0; e < C.j.size(); ++e) {
      umax = std::max(umax, U[5 * C.j[e] + q]);
      umin = std::min(umin, U[5 * C.j[e] + q]);
    }
    double alpha = 1.0;
    for (size_t e = 0; e < C.j.size(); ++e) {
      const V3 disp = (p.limiter_disp == 0) ? dv[e] : (M.r[i] + C.f_rel[e]) - ci;
      const double D = G[q][0] * disp.x + G[q][1] * disp.y + G[q][2] * disp.z;
      double psi;
      if (D > 0) psi = (umax - Ui) / D;
      else if (D < 0) psi = (umin - Ui) / D;
      else psi = 1.0;
      alpha = std::min(alpha, psi);
    }
    for (int r = 0; r < 3; ++r) G[q][r] *= alpha;
  }
}

// Time derivative of the state from its gradient (Sec. 4.1): -div F written
// with the chain rule in terms of grad U, plus w . grad U for the moving
// generator (R-pred).
void rate_chain_rule(const double U[5], const double G[5][3], const double w[3], double gamma,
                     bool moving, double dUdt[5]) {
  const double g1 = gamma - 1.0;
  const double rho = U[0];
  const double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double E = U[4];
  const double P = g1 * (E - 0.5 * rho * vv);
  double dv[3][3];   // dv[a][d] = d v_a / d x_d
  double dP[3];
  for (int d = 0; d < 3; ++d) {
    for (int a = 0; a < 3; ++a) dv[a][d] = (G[1 + a][d] - v[a] * G[0][d]) / rho;
    dP[d] = g1 * (G[4][d] - (v[0] * G[1][d] + v[1] * G[2][d] + v[2] * G[3][d]) + 0.5 * vv * G[0][d]);
  }
  const double divv = dv[0][0] + dv[1][1] + dv[2][2];
  double div[5];
  div[0] = G[1][0] + G[2][1] + G[3][2];
  for (int a = 0; a < 3; ++a) {
    double s = 0;
    for (int d = 0; d < 3; ++d) s += v[d] * G[1 + a][d];
    div[1 + a] = s + U[1 + a] * divv + dP[a];
  }
  {
    double s = 0;
    for (int d = 0; d < 3; ++d) s += v[d] * (G[4][d] + dP[d]);
    div[4] = s + (E + P) * divv;
  }
  for (int q = 0; q < 5; ++q) {
    double adv = 0;
    if (moving)
      for (int d = 0; d < 3; ++d) adv += w[d] * G[q][d];
    dUdt[q] = -div[q] + adv;
  }
}

// The same rate through the flux Jacobians J_d = dF_d/dU of the Euler
// equations: dU/dt = -sum_d J_d dU/dx_d (+ w . grad U).  Used only to check
// rate_chain_rule.
void rate_jacobian(const double U[5], const double G[5][3], const double w[3], double gamma,
                   bool moving, double dUdt[5]) {
  const double g1 = gamma - 1.0;
  const double rho = U[0];
  const double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double P = g1 * (U[4] - 0.5 * rho * vv);
  const double H = (U[4] + P) / rho;
  double out[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    double J[5][5] = {};
    // mass flux m_d
    J[0][1 + d] = 1.0;
    // momentum flux m_a v_d + P delta_ad
    for (int a = 0; a < 3; ++a) {
      J[1 + a][0] = -v[a] * v[d] + (a == d ? 0.5 * g1 * vv : 0.0);
      for (int b = 0; b < 3; ++b)
        J[1 + a][1 + b] = (a == b ? v[d] : 0.0) + (b == d ? v[a] : 0.0) - (a == d ? g1 * v[b] : 0.0);
      J[1 + a][4] = (a == d ? g1 : 0.0);
    }
    // energy flux (E + P) v_d
    J[4][0] = v[d] * (0.5 * g1 * vv - H);
    for (int b = 0; b < 3; ++b) J[4][1 + b] = (b == d ? H : 0.0) - g1 * v[b] * v[d];
    J[4][4] = gamma * v[d];
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) out[r] -= J[r][c] * G[c][d];
  }
  for (int q = 0; q < 5; ++q) {
    double adv = 0;
    if (moving)
      for (int d = 0; d < 3; ++d) adv += w[d] * G[q][d];
    dUdt[q] = out[q] + adv;
  }
}

// Face velocity (Sec. 4, item 1): normal velocity of the moving bisector at
// the face centre plus the mean velocity of the two generators.
V3 face_velocity(V3 ri, V3 rj_img, V3 wi, V3 wj, V3 f) {
  const V3 dr = rj_img - ri;
  const double len = std::sqrt(norm2(dr));
  const V3 mid = 0.5 * (ri + rj_img);
  const double s = dot(wi - wj, f - mid) / len;
  return (s / len) * dr + 0.5 * (wi + wj);
}

// Physical flux along nhat of a state given by primitives (face frame).
void phys_flux(double rho, const double v[3], double P, const double n[3], double gamma, double F[5]) {
  const double u = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  const double E = P / (gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  F[0] = rho * u;
  for (int a = 0; a < 3; ++a) F[1 + a] = rho * u * v[a] + P * n[a];
  F[4] = (E + P) * u;
}

// HLLC flux in the rest frame of the face (R-hllc; Sec. 4 item 4).
void hllc(const Prim& L, const Prim& R, const double n[3], double gamma, double F[5]) {
  const double uL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
  const double uR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
  const double cL = std::sqrt(gamma * L.P / L.rho), cR = std::sqrt(gamma * R.P / R.rho);
  const double SL = std::min(uL - cL, uR - cR);
  const double SR = std::max(uL + cL, uR + cR);
  const double Ss = (R.P - L.P + L.rho * uL * (SL - uL) - R.rho * uR * (SR - uR)) /
                    (L.rho * (SL - uL) - R.rho * (SR - uR));
  double FL[5], FR[5];
  phys_flux(L.rho, L.v, L.P, n, gamma, FL);
  phys_flux(R.rho, R.v, R.P, n, gamma, FR);
  if (SL >= 0) {
    for (int q = 0; q < 5; ++q) F[q] = FL[q];
    return;
  }
  if (SR < 0) {
    for (int q = 0; q < 5; ++q) F[q] = FR[q];
    return;
  }
  const bool left = Ss >= 0;
  const Prim& K = left ? L : R;
  const double uK = left ? uL : uR;
  const double SK = left ? SL : SR;
  const double* FK = left ? FL : FR;
  const double EK = K.P / (gamma - 1.0) + 0.5 * K.rho * (K.v[0] * K.v[0] + K.v[1] * K.v[1] + K.v[2] * K.v[2]);
  const double UK[5] = {K.rho, K.rho * K.v[0], K.rho * K.v[1], K.rho * K.v[2], EK};
  const double fac = K.rho * (SK - uK) / (SK - Ss);
  double Us[5];
  Us[0] = fac;
  for (int a = 0; a < 3; ++a) Us[1 + a] = fac * (K.v[a] + (Ss - uK) * n[a]);
  Us[4] = fac * (EK / K.rho + (Ss - uK) * (Ss + K.P / (K.rho * (SK - uK))));
  for (int q = 0; q < 5; ++q) F[q] = FK[q] + SK * (Us[q] - UK[q]);
}

// HLL flux in the rest frame of the face (Sec. 4 item 4, Toro 2009 sec. 10.3):
// one intermediate state between the fastest left- and right-going waves,
// whose average over the fan follows from the integral form of the
// conservation law.  Wave-speed bounds as in hllc().
void hll(const Prim& L, const Prim& R, const double n[3], double gamma, double F[5]) {
  const double uL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
  const double uR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
  const double cL = std::sqrt(gamma * L.P / L.rho), cR = std::sqrt(gamma * R.P / R.rho);
  const double SL = std::min(uL - cL, uR - cR);
  const double SR = std::max(uL + cL, uR + cR);
  double FL[5], FR[5];
  phys_flux(L.rho, L.v, L.P, n, gamma, FL);
  phys_flux(R.rho, R.v, R.P, n, gamma, FR);
  if (SL >= 0) {
    for (int q = 0; q < 5; ++q) F[q] = FL[q];
    return;
  }
  if (SR < 0) {
    for (int q = 0; q < 5; ++q) F[q] = FR[q];
    return;
  }
  const double EL = L.P / (gamma - 1.0) + 0.5 * L.rho * (L.v[0] * L.v[0] + L.v[1] * L.v[1] + L.v[2] * L.v[2]);
  const double ER = R.P / (gamma - 1.0) + 0.5 * R.rho * (R.v[0] * R.v[0] + R.v[1] * R.v[1] + R.v[2] * R.v[2]);
  const double UL[5] = {L.rho, L.rho * L.v[0], L.rho * L.v[1], L.rho * L.v[2], EL};
  const double UR[5] = {R.rho, R.rho * R.v[0], R.rho * R.v[1], R.rho * R.v[2], ER};
  for (int q = 0; q < 5; ++q) F[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) / (SR - SL);
}

// Lab-frame flux across a face moving with velocity wt (Sec. 4 items 3-5):
// boost both states into the face frame, solve (HLLC, or HLL when riemann
// is 1), boost the flux back.
void moving_face_flux(const double UL[5], const double UR[5], const double n[3], const double wt[3],
                      double gamma, int riemann, double F[5]) {
  Prim L = to_prim(UL, gamma), R = to_prim(UR, gamma);
  for (int a = 0; a < 3; ++a) {
    L.v[a] -= wt[a];
    R.v[a] -= wt[a];
  }
  double Ff[5];
  if (riemann == 1)
    hll(L, R, n, gamma, Ff);
  else
    hllc(L, R, n, gamma, Ff);
  const double w2 = wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2];
  F[0] = Ff[0];
  for (int a = 0; a < 3; ++a) F[1 + a] = Ff[1 + a] + wt[a] * Ff[0];
  F[4] = Ff[4] + (wt[0] * Ff[1] + wt[1] * Ff[2] + wt[2] * Ff[3]) + 0.5 * w2 * Ff[0];
}

// R-dm: the Duffell-MacFadyen factor for one face and one component.
double dm_factor(double theta, double dU, double D) {
  if (theta <= 0.0 || D == 0.0) return 1.0;
  return std::min(1.0, std::max(theta * dU / D, 0.0));
}

inline bool owns(int i, int j, int code) { return i < j || (i == j && code > 13); }

// Face geometry and the two reconstructed states of the face (i, e) of cell
// i, seen from i (Sec. 4 item 1; Sec. 4.1 reconstruction of the state at
// the face and the limiter of Duffell & MacFadyen, R-dm).  Returns the number of face floors.
struct FaceSetup {
  double UL[5], UR[5];
  double n[3];   // unit normal from i toward the neighbour image
  double wt[3];  // face velocity
  double rhoL0, rhoR0;   // densities of the face states (before any floor)
  bool fbL, fbR;         // a side fell back to its cell's half-step state
  V3 fi, fj;             // face centroid minus each side's centroid
};
int setup_face(const Mesh& M, const Params& p, int64_t i, size_t e, const double* Uh, const double* Gh,
               const double* w, FaceSetup& S) {
  const CellOut& C = M.cells[i];
  const int j = C.j[e];
  const V3 s = shift_of(M, C.code[e]);
  const V3 ri = M.r[i];
  const V3 rj = M.r[j] + s;
  const V3 ci = centroid(M, (int)i);
  const V3 cj = centroid(M, j) + s;
  const V3 f = ri + C.f_rel[e];
  const V3 dr = rj - ri;
  const double len = std::sqrt(norm2(dr));
  S.n[0] = dr.x / len;
  S.n[1] = dr.y / len;
  S.n[2] = dr.z / len;
  const V3 wi{w[3 * i], w[3 * i + 1], w[3 * i + 2]};
  const V3 wj{w[3 * j], w[3 * j + 1], w[3 * j + 2]};
  const V3 wt = face_velocity(ri, rj, wi, wj, f);
  S.wt[0] = wt.x;
  S.wt[1] = wt.y;
  S.wt[2] = wt.z;
  const V3 fi = f - ci, fj = f - cj;
  for (int q = 0; q < 5; ++q) {
    const double* gi = Gh + 15 * i + 3 * q;
    const double* gj = Gh + 15 * (int64_t)j + 3 * q;
    const double Ui = Uh[5 * i + q], Uj = Uh[5 * (int64_t)j + q];
    const double Di = gi[0] * fi.x + gi[1] * fi.y + gi[2] * fi.z;
    const double Dj = gj[0] * fj.x + gj[1] * fj.y + gj[2] * fj.z;
    S.UL[q] = Ui + dm_factor(p.theta, Uj - Ui, Di) * Di;
    S.UR[q] = Uj + dm_factor(p.theta, Ui - Uj, Dj) * Dj;
  }
  S.fi = fi;
  S.fj = fj;
  // R-floor: a side whose reconstruction needs a floor takes its cell's
  // half-step state, which the predictor has already floored.
  int hits = 0;
  double t[5];
  std::copy(S.UL, S.UL + 5, t);
  S.fbL = apply_floors(t, p) > 0;
  if (S.fbL) std::copy(Uh + 5 * i, Uh + 5 * i + 5, S.UL);
  std::copy(S.UR, S.UR + 5, t);
  S.fbR = apply_floors(t, p) > 0;
  if (S.fbR) std::copy(Uh + 5 * (int64_t)j, Uh + 5 * (int64_t)j + 5, S.UR);
  hits += S.fbL;
  hits += S.fbR;
  S.rhoL0 = S.UL[0];
  S.rhoR0 = S.UR[0];
  return hits;
}

// R-ent, the gradient of the one-component column X: the same least squares
// and S10 limiter as gradient_cell.
void gradient_scalar(const Mesh& M, const Params& p, int i, const double* X, double g[3], bool limit) {
  const CellOut& C = M.cells[i];
  const V3 ci = centroid(M, i);
  double Mm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double b[3] = {0, 0, 0};
  std::vector<V3> dv(C.j.size());
  for (size_t e = 0; e < C.j.size(); ++e) {
    const V3 d = (centroid(M, C.j[e]) + shift_of(M, C.code[e])) - ci;
    dv[e] = d;
    const double wgt = C.A[e] / norm2(d);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Mm[r][c] += wgt * comp(d, r) * comp(d, c);
    const double dX = X[C.j[e]] - X[i];
    for (int r = 0; r < 3; ++r) b[r] += wgt * dX * comp(d, r);
  }
  const double a00 = Mm[1][1] * Mm[2][2] - Mm[1][2] * Mm[2][1];
  const double a01 = Mm[0][2] * Mm[2][1] - Mm[0][1] * Mm[2][2];
  const double a02 = Mm[0][1] * Mm[1][2] - Mm[0][2] * Mm[1][1];
  const double a11 = Mm[0][0] * Mm[2][2] - Mm[0][2] * Mm[2][0];
  const double a12 = Mm[0][2] * Mm[1][0] - Mm[0][0] * Mm[1][2];
  const double a22 = Mm[0][0] * Mm[1][1] - Mm[0][1] * Mm[1][0];
  const double det = Mm[0][0] * a00 + Mm[0][1] * (Mm[1][2] * Mm[2][0] - Mm[1][0] * Mm[2][2]) +
                     Mm[0][2] * (Mm[1][0] * Mm[2][1] - Mm[1][1] * Mm[2][0]);
  const double inv[3][3] = {{a00 / det, a01 / det, a02 / det},
                            {a01 / det, a11 / det, a12 / det},
                            {a02 / det, a12 / det, a22 / det}};
  for (int r = 0; r < 3; ++r) g[r] = inv[r][0] * b[0] + inv[r][1] * b[1] + inv[r][2] * b[2];
  if (!limit) return;
  double xmax = X[i], xmin = X[i];
  for (size_t e = 0; e < C.j.size(); ++e) {
    xmax = std::max(xmax, X[C.j[e]]);
    xmin = std::min(xmin, X[C.j[e]]);
  }
  double alpha = 1.0;
  for (size_t e = 0; e < C.j.size(); ++e) {
    const V3 disp = (p.limiter_disp == 0) ? dv[e] : (M.r[i] + C.f_rel[e]) - ci;
    const double D = g[0] * disp.x + g[1] * disp.y + g[2] * disp.z;
    double psi;
    if (D > 0) psi = (xmax - X[i]) / D;
    else if (D < 0) psi = (xmin - X[i]) / D;
    else psi = 1.0;
    alpha = std::min(alpha, psi);
  }
  for (int r = 0; r < 3; ++r) g[r] *= alpha;
}

// R-ent, time derivative of X = rho A for the predictor: -div(X v), plus
// w . grad X for the moving generator (R-pred).
double rate_entropy(const double U[5], const double G[5][3], double X, const double gX[3], const double w[3],
                    bool moving) {
  const double rho = U[0];
  const double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  double divv = 0;
  for (int a = 0; a < 3; ++a) divv += (G[1 + a][a] - v[a] * G[0][a]) / rho;
  double r = -(v[0] * gX[0] + v[1] * gX[1] + v[2] * gX[2] + X * divv);
  if (moving) r += w[0] * gX[0] + w[1] * gX[1] + w[2] * gX[2];
  return r;
}

// R-ent, the face-frame flux of X and the face's shock Mach number, for the
// face-frame primitive states L, R (after the face floors) and the entropic
// functions A_L, A_R of the two sides.
void entropy_face(const Prim& L, const Prim& R, const double n[3], double gamma, int riemann, double AL, double AR,
                  double& FX, double& mach) {
  const double uL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
  const double uR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
  const double cL = std::sqrt(gamma * L.P / L.rho), cR = std::sqrt(gamma * R.P / R.rho);
  const double SL = std::min(uL - cL, uR - cR);
  const double SR = std::max(uL + cL, uR + cR);
  const double Ss = (R.P - L.P + L.rho * uL * (SL - uL) - R.rho * uR * (SR - uR)) /
                    (L.rho * (SL - uL) - R.rho * (SR - uR));
  const double ps = L.P + L.rho * (SL - uL) * (Ss - uL);
  const double k = (gamma + 1.0) / (2.0 * gamma);
  const double ML = std::sqrt(1.0 + k * std::max(0.0, ps / L.P - 1.0));
  const double MR = std::sqrt(1.0 + k * std::max(0.0, ps / R.P - 1.0));
  mach = std::max(ML, MR);
  const double XL = L.rho * AL, XR = R.rho * AR;
  if (SL >= 0) {
    FX = XL * uL;
  } else if (SR < 0) {
    FX = XR * uR;
  } else if (riemann == 1) {
    FX = (SR * XL * uL - SL * XR * uR + SL * SR * (XR - XL)) / (SR - SL);
  } else {
    // HLLC: the star-region mass flux carries the entropic function of the
    // side the contact leaves behind.
    double F[5];
    hllc(L, R, n, gamma, F);
    FX = F[0] * (Ss >= 0 ? AL : AR);
  }
}

// Fluxes of all faces and their accumulation into dQ (Sec. 4, update of the
// charges and items 1-5).  Each face's flux is computed once, by the cell
// with the lower index, with that cell's face geometry; R-upd fixes the
// signs.
// With the entropy column (Xh, gXh non-null, R-ent) also the flux of X into
// dS and each cell's largest face Mach number into mach.
int fluxes(const Mesh& M, const Params& p, const double* Uh, const double* Gh, const double* w, double dt,
           double* dQ, int64_t* face_hits, const double* Xh = nullptr, const double* gXh = nullptr,
           double* dS = nullptr, double* mach = nullptr) {
  const int64_t n = M.n;
  const bool ent = Xh != nullptr;
  std::vector<std::vector<std::array<double, 5>>> phi(n);
  std::vector<std::vector<double>> phiX(ent ? n : 0), machF(ent ? n : 0);
  int64_t hits = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : hits)
  for (int64_t i = 0; i < n; ++i) {
    const CellOut& C = M.cells[i];
    phi[i].assign(C.j.size(), {0, 0, 0, 0, 0});
    if (ent) {
      phiX[i].assign(C.j.size(), 0.0);
      machF[i].assign(C.j.size(), 0.0);
    }
    for (size_t e = 0; e < C.j.size(); ++e) {
      if (!owns((int)i, C.j[e], C.code[e])) continue;
      FaceSetup S;
      hits += setup_face(M, p, i, e, Uh, Gh, w, S);
      double F[5];
      moving_face_flux(S.UL, S.UR, S.n, S.wt, p.gamma, p.riemann, F);
      for (int q = 0; q < 5; ++q) phi[i][e][q] = dt * C.A[e] * F[q];
      if (ent) {
        const int j = C.j[e];
        const double* gi = gXh + 3 * i;
        const double* gj = gXh + 3 * (int64_t)j;
        const double Di = gi[0] * S.fi.x + gi[1] * S.fi.y + gi[2] * S.fi.z;
        const double Dj = gj[0] * S.fj.x + gj[1] * S.fj.y + gj[2] * S.fj.z;
        const double XL = S.fbL ? Xh[i] : Xh[i] + dm_factor(p.theta, Xh[j] - Xh[i], Di) * Di;
        const double XR = S.fbR ? Xh[j] : Xh[j] + dm_factor(p.theta, Xh[i] - Xh[j], Dj) * Dj;
        Prim L = to_prim(S.UL, p.gamma), R = to_prim(S.UR, p.gamma);
        for (int a = 0; a < 3; ++a) {
          L.v[a] -= S.wt[a];
          R.v[a] -= S.wt[a];
        }
        double FX, mf;
        entropy_face(L, R, S.n, p.gamma, p.riemann, XL / S.rhoL0, XR / S.rhoR0, FX, mf);
        phiX[i][e] = dt * C.A[e] * FX;
        machF[i][e] = mf;
      }
    }
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    const CellOut& C = M.cells[i];
    double acc[5] = {0, 0, 0, 0, 0};
    double accX = 0.0, mx = 0.0;
    for (size_t e = 0; e < C.j.size(); ++e) {
      const int j = C.j[e];
      if (owns((int)i, j, C.code[e])) {
        for (int q = 0; q < 5; ++q) acc[q] -= phi[i][e][q];
        if (ent) {
          accX -= phiX[i][e];
          mx = std::max(mx, machF[i][e]);
        }
      } else {
        const CellOut& D = M.cells[j];
        const int want = kneg(C.code[e]);
        size_t e2 = D.j.size();
        for (size_t t = 0; t < D.j.size(); ++t)
          if (D.j[t] == (int)i && D.code[t] == want) { e2 = t; break; }
        if (e2 == D.j.size()) { bad++; continue; }
        for (int q = 0; q < 5; ++q) acc[q] += phi[j][e2][q];
        if (ent) {
          accX += phiX[j][e2];
          mx = std::max(mx, machF[j][e2]);
        }
      }
    }
    for (int q = 0; q < 5; ++q) dQ[5 * i + q] = acc[q];
    if (ent) {
      dS[i] = accX;
      mach[i] = mx;
    }
  }
  if (face_hits) *face_hits = hits;
  return bad ? 2 : 0;
}

}  // namespace

// ===========================================================================
// C ABI for the Python test harness.
// ===========================================================================
extern "C" {

typedef Params orc_params;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// method: 0 brute force, 1 grid.  want_cert: compute the non-degeneracy
// margin.  exhaustive: brute force without the farthest-vertex skip.
void* orc_mesh_build(int64_t n, const double* pos, const double* box, int32_t method, int32_t want_cert,
                     int32_t exhaustive) {
  Mesh* M = new Mesh();
  M->n = n;
  M->L = {box[0], box[1], box[2]};
  M->r.resize(n);
  for (int64_t i = 0; i < n; ++i) M->r[i] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  M->cells.resize(n);
  Grid G;
  if (method == 1) G = make_grid(*M, 8.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    if (method == 1) build_cell_grid(*M, G, (int)i, M->cells[i], want_cert != 0);
    else build_cell_brute(*M, (int)i, exhaustive != 0, M->cells[i]);
  }
  for (int64_t i = 0; i < n; ++i) {
    if (M->cells[i].delta == M->cells[i].delta) M->delta_min = std::min(M->delta_min, M->cells[i].delta);
    if (M->cells[i].status) M->status = 1;
  }
  return M;
}

// Only the cells listed in idx (grid path, with certificate); the other
// cells are left empty.  For sampled checks on large point sets.
void* orc_mesh_build_subset(int64_t n, const double* pos, const double* box, const int64_t* idx, int64_t m) {
  Mesh* M = new Mesh();
  M->n = n;
  M->L = {box[0], box[1], box[2]};
  M->r.resize(n);
  for (int64_t i = 0; i < n; ++i) M->r[i] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  M->cells.resize(n);
  const Grid G = make_grid(*M, 8.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < m; ++t) build_cell_grid(*M, G, (int)idx[t], M->cells[idx[t]], true);
  for (int64_t t = 0; t < m; ++t) {
    const CellOut& C = M->cells[idx[t]];
    if (C.delta == C.delta) M->delta_min = std::min(M->delta_min, C.delta);
    if (C.status) M->status = 1;
  }
  return M;
}

void orc_mesh_free(void* m) { delete (Mesh*)m; }
int32_t orc_mesh_status(void* m) { return ((Mesh*)m)->status; }
double orc_mesh_delta_min(void* m) { return ((Mesh*)m)->delta_min; }

int64_t orc_mesh_nfaces(void* m) {
  const Mesh* M = (Mesh*)m;
  int64_t s = 0;
  for (const CellOut& C : M->cells) s += (int64_t)C.j.size();
  return s;
}

// Per-cell geometry: V, centroid (absolute), tetrahedral volume, farthest
// vertex distance, vertex count, non-degeneracy margin.
void orc_mesh_cells(void* m, double* V, double* c, double* vtet, double* rmax, int32_t* nvert, double* delta) {
  const Mesh* M = (Mesh*)m;
  for (int64_t i = 0; i < M->n; ++i) {
    const CellOut& C = M->cells[i];
    V[i] = C.V;
    const V3 cc = M->r[i] + C.c_rel;
    c[3 * i] = cc.x;
    c[3 * i + 1] = cc.y;
    c[3 * i + 2] = cc.z;
    vtet[i] = C.vtet;
    rmax[i] = C.rmax;
    nvert[i] = C.nvert;
    delta[i] = C.delta;
  }
}

// Directed faces of every cell, ordered by (cell, neighbour, image code):
// off[n+1], j, image code, area, face centroid (absolute; may lie outside
// the box when the face is across the periodic boundary).
void orc_mesh_faces(void* m, int64_t* off, int32_t* j, int32_t* code, double* A, double* f) {
  const Mesh* M = (Mesh*)m;
  int64_t t = 0;
  for (int64_t i = 0; i < M->n; ++i) {
    off[i] = t;
    const CellOut& C = M->cells[i];
    for (size_t e = 0; e < C.j.size(); ++e, ++t) {
      j[t] = C.j[e];
      code[t] = C.code[e];
      A[t] = C.A[e];
      const V3 ff = M->r[i] + C.f_rel[e];
      f[3 * t] = ff.x;
      f[3 * t + 1] = ff.y;
      f[3 * t + 2] = ff.z;
    }
  }
  off[M->n] = t;
}

// Initial charges from primitives (Sec. 4.3): Q_i = U(prim_i) V_i.
void orc_init_charges(void* m, const orc_params* p, const double* prim, double* Q) {
  const Mesh* M = (Mesh*)m;
  for (int64_t i = 0; i < M->n; ++i) {
    const double* w = prim + 5 * i;
    const double V = M->cells[i].V;
    const double rho = w[0];
    const double ke = 0.5 * rho * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    Q[5 * i] = rho * V;
    for (int a = 0; a < 3; ++a) Q[5 * i + 1 + a] = rho * w[1 + a] * V;
    Q[5 * i + 4] = (w[4] / (p->gamma - 1.0) + ke) * V;
  }
}

// Cell state at the start of a step (Sec. 4, charges; Sec. 4.1 floors;
// Sec. 4.2 mesh velocity and timestep).  Returns dt_cfl = min_i dt_i.
double orc_cell_state(void* m, const orc_params* p, const double* Q, double* U, double* w, double* dti,
                      int64_t* hits) {
  const Mesh* M = (Mesh*)m;
  int64_t h = 0;
  double dtmin = 1e300;
  for (int64_t i = 0; i < M->n; ++i) {
    const double V = M->cells[i].V;
    for (int q = 0; q < 5; ++q) U[5 * i + q] = Q[5 * i + q] / V;
    h += apply_floors(U + 5 * i, *p) > 0;
    mesh_velocity(*M, *p, (int)i, U + 5 * i, w + 3 * i, dti[i]);
    dtmin = std::min(dtmin, dti[i]);
  }
  if (hits) *hits = h;
  return dtmin;
}

void orc_gradient(void* m, const orc_params* p, const double* U, double* G, int32_t limit) {
  const Mesh* M = (Mesh*)m;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < M->n; ++i) {
    double g[5][3];
    gradient_cell(*M, *p, (int)i, U, g, limit != 0);
    for (int q = 0; q < 5; ++q)
      for (int r = 0; r < 3; ++r) G[15 * i + 3 * q + r] = g[q][r];
  }
}

// Half-step predictor (Sec. 4.1): U^(n+1/2) = U^n + dt/2 dU/dt, then floors.
// form 0: chain rule, form 1: explicit flux Jacobians.
void orc_predict(void* m, const orc_params* p, const double* U, const double* G, const double* w, double dt,
                 double* Uh, int32_t form, int64_t* hits) {
  const Mesh* M = (Mesh*)m;
  int64_t h = 0;
  for (int64_t i = 0; i < M->n; ++i) {
    double g[5][3], r[5];
    for (int q = 0; q < 5; ++q)
      for (int c = 0; c < 3; ++c) g[q][c] = G[15 * i + 3 * q + c];
    const bool moving = p->predictor_frame == 0;
    if (form == 0) rate_chain_rule(U + 5 * i, g, w + 3 * i, p->gamma, moving, r);
    else rate_jacobian(U + 5 * i, g, w + 3 * i, p->gamma, moving, r);
    for (int q = 0; q < 5; ++q) Uh[5 * i + q] = U[5 * i + q] + 0.5 * dt * r[q];
    h += apply_floors(Uh + 5 * i, *p) > 0;
  }
  if (hits) *hits = h;
}

// Reconstructed face states of every directed face, as seen from its cell:
// UL on the cell's side, UR on the neighbour's side; plus normal and face
// velocity.  Arrays are indexed like orc_mesh_faces.
void orc_face_states(void* m, const orc_params* p, const double* Uh, const double* Gh, const double* w, double* UL,
                     double* UR, double* nrm, double* wt) {
  const Mesh* M = (Mesh*)m;
  int64_t t = 0;
  for (int64_t i = 0; i < M->n; ++i)
    for (size_t e = 0; e < M->cells[i].j.size(); ++e, ++t) {
      FaceSetup S;
      setup_face(*M, *p, i, e, Uh, Gh, w, S);
      for (int q = 0; q < 5; ++q) {
        UL[5 * t + q] = S.UL[q];
        UR[5 * t + q] = S.UR[q];
      }
      for (int a = 0; a < 3; ++a) {
        nrm[3 * t + a] = S.n[a];
        wt[3 * t + a] = S.wt[a];
      }
    }
}

int32_t orc_fluxes(void* m, const orc_params* p, const double* Uh, const double* Gh, const double* w, double dt,
                   double* dQ, int64_t* hits) {
  return fluxes(*(Mesh*)m, *p, Uh, Gh, w, dt, dQ, hits);
}

// The step, with the entropy column when S is non-null (R-ent); mach_out
// (optional) receives each cell's largest face Mach number.
static int32_t step_impl(int64_t n, double* pos, double* Q, double* S, double* w_out, const orc_params* p,
                         double dt_max, int32_t method, double* dt_out, int64_t* counters, double* mach_out) {
  if (S && p->half_step_mesh) return 3;   // the two options are not combined
  void* mh = orc_mesh_build(n, pos, p->box, method, 0, 0);
  Mesh* M = (Mesh*)mh;
  if (M->status) { delete M; return 1; }
  std::vector<double> U(5 * n), Uh(5 * n), G(15 * n), Gh(15 * n), dti(n), dQ(5 * n);
  int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  double dt = orc_cell_state(mh, p, Q, U.data(), w_out, dti.data(), &c0);
  dt = std::min(dt, dt_max);
  orc_gradient(mh, p, U.data(), G.data(), p->limit_mask & 1);
  orc_predict(mh, p, U.data(), G.data(), w_out, dt, Uh.data(), 0, &c1);
  // R-ent: X = S / V, its gradient and its half-step value.
  std::vector<double> X, Xh, gX, gXh, dS, mach;
  if (S) {
    X.resize(n); Xh.resize(n); gX.resize(3 * n); gXh.resize(3 * n); dS.resize(n); mach.resize(n);
    for (int64_t i = 0; i < n; ++i) X[i] = S[i] / M->cells[i].V;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      gradient_scalar(*M, *p, (int)i, X.data(), &gX[3 * i], p->limit_mask & 1);
      double g[5][3];
      for (int q = 0; q < 5; ++q)
        for (int c = 0; c < 3; ++c) g[q][c] = G[15 * i + 3 * q + c];
      Xh[i] = X[i] + 0.5 * dt * rate_entropy(&U[5 * i], g, X[i], &gX[3 * i], w_out + 3 * i,
                                             p->predictor_frame == 0);
    }
  }
  // R-tess: the second half of the step works on the mesh of the generators
  // moved to the half step.
  Mesh* F = M;
  if (p->half_step_mesh) {
    std::vector<double> ph(3 * n);
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        double x = pos[3 * i + a] + w_out[3 * i + a] * (0.5 * dt);
        if (x < 0) x += p->box[a];
        if (x >= p->box[a]) x -= p->box[a];
        ph[3 * i + a] = x;
      }
    F = (Mesh*)orc_mesh_build(n, ph.data(), p->box, method, 0, 0);
    if (F->status) { delete F; delete M; return 1; }
  }
  orc_gradient(F, p, Uh.data(), Gh.data(), (p->limit_mask >> 1) & 1);
  if (S) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
      gradient_scalar(*F, *p, (int)i, Xh.data(), &gXh[3 * i], (p->limit_mask >> 1) & 1);
  }
  const int rc = S ? fluxes(*F, *p, Uh.data(), Gh.data(), w_out, dt, dQ.data(), &c2, Xh.data(), gXh.data(),
                            dS.data(), mach.data())
                   : fluxes(*F, *p, Uh.data(), Gh.data(), w_out, dt, dQ.data(), &c2);
  if (rc) {
    if (F != M) delete F;
    delete M;
    return rc;
  }
  const double g = p->gamma, g1 = p->gamma - 1.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int q = 0; q < 5; ++q) Q[5 * i + q] += dQ[5 * i + q];
    // Floors at the cell centre after the step, with the volume of the mesh
    // the fluxes used (time n, or the half step under R-tess).
    const double V = F->cells[i].V;
    bool from_entropy = false;
    if (S) {
      S[i] += dS[i];
      if (mach_out) mach_out[i] = mach[i];
      if (mach[i] < p->mach_threshold) {
        // R-ent: no shock at this cell: the pressure follows the entropy.
        const double m = Q[5 * i];
        const double A = S[i] / m;
        const double P = A * std::pow(m / V, g);
        const double p2 = Q[5 * i + 1] * Q[5 * i + 1] + Q[5 * i + 2] * Q[5 * i + 2] + Q[5 * i + 3] * Q[5 * i + 3];
        Q[5 * i + 4] = P * V / g1 + 0.5 * p2 / m;
        from_entropy = true;
      }
    }
    double Ui[5];
    for (int q = 0; q < 5; ++q) Ui[q] = Q[5 * i + q] / V;
    const bool floored = apply_floors(Ui, *p) != 0;
    if (floored) {
      c3++;
      for (int q = 0; q < 5; ++q) Q[5 * i + q] = Ui[q] * V;
    }
    if (S && (!from_entropy || floored)) {
      // R-ent: the energy was integrated (or floored): the entropy follows
      // the new state.
      const Prim pr = to_prim(Ui, g);
      S[i] = Q[5 * i] * pr.P / std::pow(pr.rho, g);
    }
    // Drift by a full step with periodic wrap (Sec. 2, item 5).
    for (int a = 0; a < 3; ++a) {
      double x = pos[3 * i + a] + w_out[3 * i + a] * dt;
      if (x < 0) x += p->box[a];
      if (x >= p->box[a]) x -= p->box[a];
      pos[3 * i + a] = x;
    }
  }
  if (dt_out) *dt_out = dt;
  if (counters) {
    counters[0] = c0;
    counters[1] = c1;
    counters[2] = c2;
    counters[3] = c3;
  }
  if (F != M) delete F;
  delete M;
  return 0;
}

// One whole step (Sec. 2 outline).  pos, Q in/out; w_out receives the mesh
// velocities used.  counters: [0] cell floors at the start, [1] predictor
// floors, [2] face floors, [3] floors after the update.  Returns 0, or a
// non-zero code when the tessellation or the face topology failed.
int32_t orc_step(int64_t n, double* pos, double* Q, double* w_out, const orc_params* p, double dt_max,
                 int32_t method, double* dt_out, int64_t* counters) {
  return step_impl(n, pos, Q, nullptr, w_out, p, dt_max, method, dt_out, counters, nullptr);
}

// As orc_step with the entropy charge S = m A (R-ent, Sec. 4.3) in/out and
// each cell's largest face Mach number out (mach may be NULL).  Returns 3
// when combined with the half-step mesh.
int32_t orc_step_entropy(int64_t n, double* pos, double* Q, double* S, double* w_out, const orc_params* p,
                         double dt_max, int32_t method, double* dt_out, int64_t* counters, double* mach) {
  return step_impl(n, pos, Q, S, w_out, p, dt_max, method, dt_out, counters, mach);
}

// Entropy charges S = m P rho^-gamma of primitive states on a mesh (R-ent).
void orc_init_entropy(void* m, const orc_params* p, const double* prim, double* S) {
  const Mesh* M = (Mesh*)m;
  for (int64_t i = 0; i < M->n; ++i) {
    const double rho = prim[5 * i], P = prim[5 * i + 4];
    S[i] = rho * M->cells[i].V * P / std::pow(rho, p->gamma);
  }
}

void orc_face_velocity(const double* ri, const double* rj_img, const double* wi, const double* wj, const double* f,
                       double* wt) {
  const V3 r = face_velocity({ri[0], ri[1], ri[2]}, {rj_img[0], rj_img[1], rj_img[2]}, {wi[0], wi[1], wi[2]},
                             {wj[0], wj[1], wj[2]}, {f[0], f[1], f[2]});
  wt[0] = r.x;
  wt[1] = r.y;
  wt[2] = r.z;
}

// Lab-frame flux of conserved states UL, UR across a face with unit normal n
// moving with velocity wt; riemann 0 is HLLC, 1 is HLL.
void orc_moving_face_flux(const double* UL, const double* UR, const double* n, const double* wt, double gamma,
                          int32_t riemann, double* F) {
  moving_face_flux(UL, UR, n, wt, gamma, riemann, F);
}

// R-ent: flux of X = rho A and shock Mach number of a face-frame Riemann
// problem on primitive states (riemann 0 HLLC, 1 HLL).
void orc_entropy_face(const double* WL, const double* WR, const double* n, double gamma, int32_t riemann,
                      double AL, double AR, double* FX, double* mach) {
  Prim L{WL[0], {WL[1], WL[2], WL[3]}, WL[4]};
  Prim R{WR[0], {WR[1], WR[2], WR[3]}, WR[4]};
  entropy_face(L, R, n, gamma, riemann, AL, AR, *FX, *mach);
}

// HLL in the face frame on primitive states (rho, vx, vy, vz, P).
void orc_hll_prim(const double* WL, const double* WR, const double* n, double gamma, double* F) {
  Prim L{WL[0], {WL[1], WL[2], WL[3]}, WL[4]};
  Prim R{WR[0], {WR[1], WR[2], WR[3]}, WR[4]};
  hll(L, R, n, gamma, F);
}

// HLLC in the face frame on primitive states (rho, vx, vy, vz, P).
void orc_hllc_prim(const double* WL, const double* WR, const double* n, double gamma, double* F) {
  Prim L{WL[0], {WL[1], WL[2], WL[3]}, WL[4]};
  Prim R{WR[0], {WR[1], WR[2], WR[3]}, WR[4]};
  hllc(L, R, n, gamma, F);
}

double orc_dm_factor(double theta, double dU, double D) { return dm_factor(theta, dU, D); }

int32_t orc_apply_floors(const orc_params* p, double* U) { return apply_floors(U, *p); }

// ---------------------------------------------------------------------------
// Exact solution of the 1-D Riemann problem for an ideal gas (the textbook
// solver the paper's Riemann solvers follow, Toro 2009, ch. 4): the star
// pressure is the root of f_L(p) + f_R(p) + u_R - u_L, found by bisection
// (f is increasing in p), then the self-similar solution is sampled at
// xi = x/t.  W = (rho, u, p).
// ---------------------------------------------------------------------------
static double pfun(double p, double rho, double pk, double gamma) {
  const double c = std::sqrt(gamma * pk / rho);
  if (p > pk) {
    const double A = 2.0 / ((gamma + 1.0) * rho);
    const double B = (gamma - 1.0) / (gamma + 1.0) * pk;
    return (p - pk) * std::sqrt(A / (p + B));
  }
  return 2.0 * c / (gamma - 1.0) * (std::pow(p / pk, (gamma - 1.0) / (2.0 * gamma)) - 1.0);
}

int32_t orc_exact_riemann(const double* WL, const double* WR, double gamma, int64_t m, const double* xi, double* W,
                          double* star) {
  const double rL = WL[0], uL = WL[1], pL = WL[2];
  const double rR = WR[0], uR = WR[1], pR = WR[2];
  const double cL = std::sqrt(gamma * pL / rL), cR = std::sqrt(gamma * pR / rR);
  if (2.0 * (cL + cR) / (gamma - 1.0) <= uR - uL) return 1;   // vacuum generated
  auto f = [&](double p) { return pfun(p, rL, pL, gamma) + pfun(p, rR, pR, gamma) + uR - uL; };
  double lo = 1e-300, hi = std::max(pL, pR);
  while (f(hi) < 0) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (f(mid) < 0) lo = mid;
    else hi = mid;
  }
  const double ps = 0.5 * (lo + hi);
  const double us = 0.5 * (uL + uR) + 0.5 * (pfun(ps, rR, pR, gamma) - pfun(ps, rL, pL, gamma));
  star[0] = ps;
  star[1] = us;
  const double g = gamma;
  const double G6 = (g - 1.0) / (g + 1.0);
  for (int64_t t = 0; t < m; ++t) {
    const double s = xi[t];
    double r, u, pp;
    if (s <= us) {   // left of the contact
      if (ps > pL) {
        const double SL = uL - cL * std::sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g));
        if (s <= SL) { r = rL; u = uL; pp = pL; }
        else { r = rL * (ps / pL + G6) / (G6 * ps / pL + 1.0); u = us; pp = ps; }
      } else {
        const double SHL = uL - cL;
        const double cs = cL * std::pow(ps / pL, (g - 1.0) / (2.0 * g));
        const double STL = us - cs;
        if (s <= SHL) { r = rL; u = uL; pp = pL; }
        else if (s > STL) { r = rL * std::pow(ps / pL, 1.0 / g); u = us; pp = ps; }
        else {
          u = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + s);
          const double c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (uL - s));
          r = rL * std::pow(c / cL, 2.0 / (g - 1.0));
          pp = pL * std::pow(c / cL, 2.0 * g / (g - 1.0));
        }
      }
    } else {         // right of the contact
      if (ps > pR) {
        const double SR = uR + cR * std::sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g));
        if (s >= SR) { r = rR; u = uR; pp = pR; }
        else { r = rR * (ps / pR + G6) / (G6 * ps / pR + 1.0); u = us; pp = ps; }
      } else {
        const double SHR = uR + cR;
        const double cs = cR * std::pow(ps / pR, (g - 1.0) / (2.0 * g));
        const double STR = us + cs;
        if (s >= SHR) { r = rR; u = uR; pp = pR; }
        else if (s < STR) { r = rR * std::pow(ps / pR, 1.0 / g); u = us; pp = ps; }
        else {
          u = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + s);
          const double c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (uR - s));
          r = rR * std::pow(c / cR, 2.0 / (g - 1.0));
          pp = pR * std::pow(c / cR, 2.0 * g / (g - 1.0));
        }
      }
    }
    W[3 * t] = r;
    W[3 * t + 1] = u;
    W[3 * t + 2] = pp;
  }
  return 0;
}

}  // extern "C"
