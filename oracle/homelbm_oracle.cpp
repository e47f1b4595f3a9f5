// homelbm_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
//
// A plain, slow, scalar CPU implementation of the HOME-LBM D3Q27 time step
// ("the oracle").  Only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it.  It shares no code with the GPU library:
// it reconstructs, streams and projects the 27 distributions explicitly, one
// cell and one direction at a time, in the scalar type it is instantiated with
// (double by default; std::complex<double> for complex-step derivatives; float
// to measure the intrinsic single-precision floor).
//
// Source: "High-Performance Moment-Encoded Lattice Boltzmann Method with
// Stability-Guided Quantization" (arXiv 2602.05295).
//   moments                  Sec. 3.1, Eq. (rho_u_stress)
//   reconstruction h         Sec. 3.2, Eq. (three_order_f)
//   moment-space collision   App. A, Eqs. (ourmomentcollision_*)
//   step order               Sec. 4.2, Alg. 2 (collide -> reconstruct f+ ->
//                            pull-stream f_i(x) = f+_i(x - c_i) -> project)
//   moment boundary at p     Sec. 3.2, "Solid coupling" (rho^p = rho^x,
//                            S^p = u^p u^p + (S^x - u^x u^x))
//   16-bit codec             Sec. 5.3 (moment ranges, range reduction of rho S,
//                            normalisation, b-bit quantisation, dithering)
//
// Readings taken where the paper is silent, ambiguous or garbled:
//   R1  Third-order term.  The six (alpha alpha beta) terms carry 1/(2 cs^6);
//       the xyz term carries 1/cs^6, which is what the orthogonal Hermite
//       projection gives (the xyz index triple has six permutations, the others
//       three).  literal_xyz = 1 uses the printed 1/(2 cs^6) for xyz as well.
//   R2  S is the Hermite second moment, rho S = sum (c c - cs^2 delta) f, so
//       its equilibrium is u u.  The 16-bit form stores N = rho S - rho u u.
//   R3  The 16-bit form stores u (range [-0.4, 0.4]), not rho u.
//   R4  The stored state is the post-stream (pre-collision) moments.
//   R5  Codes outside [0, 2^b - 1] saturate.
//   R6  The dither is drawn per (cell, step, component) from a counter-based
//       hash (pcg_hash of Jarzynski & Olano, JCGT 2020), sliced into 6-bit
//       fields: xi = (v + 1/2)/64 - 1/2, an exactly zero-mean uniform on
//       (-1/2, 1/2).  Mode 2 keeps one spatial pattern for all steps.
//   R7  D3Q27 lattice: c_i in {-1,0,1}^3, tensor-product weights from
//       w1(0) = 2/3, w1(+-1) = 1/6; i = (cx+1) + 3(cy+1) + 9(cz+1).
//   R8  Bulk: App. A resets the trace of S to |u|^2 (rate 1).
//   R9  nu = cs^2 (tau - 1/2).
//   R10 Walls: halfway bounce-back on a voxel mask, f_i(x) = f+_opp(i)(x)
//       when x - c_i is solid.  Solid cells hold the rest state.
//   R11 Open faces (inflow = 1): at x = 0 the links with c_x = +1 take the
//       moment boundary of Sec. 3.2 with p on the face, u^p = u_in and the
//       post-collision moments of x; at x = nx-1 the links with c_x = -1 take
//       f+_i(nx-1, y - c_y, z - c_z) (zero gradient).  y and z are periodic.
//       The face rule is applied before the solid rule.
//   R12 Body force: the stored momentum includes F/2 (Eq. rho_u_stress) and
//       the collision follows App. A with its force terms.
//   R15 The encode decision q = floor(m' (2^b - 1) + 1/2 + xi) is taken in
//       double precision from the double-precision step, half-way values
//       rounding up, as printed.  (A single-precision implementation meets
//       the same decision to within one code.)
//   R16 Wall rule 1 (the solid coupling of Sec. 3.2 on a voxel mask): the
//       link from fluid x to its solid source s = x - c_i meets the solid at
//       the link midpoint p = x - c_i/2; f_i(x) = h_i(rho^p, u^p, S^p) with
//       rho^p = rho^x, u^p = V + W x (p - C) of the object s belongs to (mask
//       value = object id, positions taken from x without wrapping) and
//       S^p = u^p u^p + (S^x - u^x u^x), x's post-collision moments.  Wall
//       rule 0 is R10.
//   R26 Wall rule 2 (the solid coupling of Sec. 3.2 with the obstacles'
//       triangle meshes, as the paper's per-triangle solid correction finds
//       it): which links to replace is still decided by the mask (fluid x,
//       solid s = x - c_i); p is the point where the link segment from x to
//       x - c_i first meets a triangle (nearest to x, ties to the lowest
//       triangle index, edges included), and u^p is taken there from the
//       triangle's object.  A link that meets no triangle is not coupled: it
//       keeps the pull from its resting solid source.  With objects at rest
//       u^p = 0 wherever p lies, so where every solid link meets a mesh rules
//       1 and 2 then agree.
//   R18 Bit allocation b_rho_u / b_S: the codes of rho and u take b1 bits,
//       those of N b2 bits (same ranges, rounding and dither), concatenated
//       low bit first, rho, ux, uy, uz, Nxx, Nyy, Nzz, Nxy, Nxz, Nyz, into
//       ceil((4 b1 + 6 b2)/32) words; 16/16 is the paired layout above.
//   R17 Force and torque on an object: momentum exchange over its links,
//       -(f_i(x) + f+_opp(i)(x)) c_i per link and step (the momentum the
//       link's outgoing and returning distributions deliver to the solid),
//       torque (p - C) x that, summed over the object's links.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double CS2 = 1.0 / 3.0;  // lattice sound speed squared, Sec. 3.2

struct Lattice {
  int c[27][3];
  double cd[27][3];
  double w[27];
  int opp[27];
  Lattice() {
    const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy)
        for (int cx = -1; cx <= 1; ++cx) {
          const int i = (cx + 1) + 3 * (cy + 1) + 9 * (cz + 1);
          c[i][0] = cx;
          c[i][1] = cy;
          c[i][2] = cz;
          w[i] = w1[cx + 1] * w1[cy + 1] * w1[cz + 1];
        }
    for (int i = 0; i < 27; ++i) {
      for (int a = 0; a < 3; ++a) cd[i][a] = double(c[i][a]);
      for (int k = 0; k < 27; ++k)
        if (c[k][0] == -c[i][0] && c[k][1] == -c[i][1] && c[k][2] == -c[i][2]) opp[i] = k;
    }
  }
};
const Lattice LAT;

inline double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

// One cell in the paper's variables: density, velocity, second-order tensor S
// (stored as a full symmetric 3x3 array for plainness).
template <class T>
struct Cell {
  T rho;
  T u[3];
  T S[3][3];
};

// Stored-moment order used throughout: rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz
// with j = rho u and P = rho S.
const int PA[6] = {0, 1, 2, 0, 0, 1};
const int PB[6] = {0, 1, 2, 1, 2, 2};

// The seven third-order index triples of Eq. (three_order_f):
// xxy, xyy, xxz, xzz, yzz, yyz, xyz.
const int T3[7][3] = {{0, 0, 1}, {0, 1, 1}, {0, 0, 2}, {0, 2, 2}, {1, 2, 2}, {1, 1, 2}, {0, 1, 2}};

// Hermite reconstruction h_i(rho, u, S), Eq. (three_order_f).  Every constant
// is cast to T so that the float instantiation computes in float.
template <class T>
T hermite_f(int i, const Cell<T>& q, bool literal_xyz) {
  const double* c = LAT.cd[i];
  // first order: c.u / cs^2
  T first = T(c[0]) * q.u[0] + T(c[1]) * q.u[1] + T(c[2]) * q.u[2];
  first = first * T(1.0 / CS2);
  // second order: H2(c) : S / (2 cs^4), full contraction over alpha, beta
  T second = T(0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) second = second + T(c[a] * c[b] - CS2 * kd(a, b)) * q.S[a][b];
  second = second * T(1.0 / (2.0 * CS2 * CS2));
  // third order: sum over the seven triples of coef * H3_abg(c) * T_abg
  T third = T(0.0);
  for (int k = 0; k < 7; ++k) {
    const int a = T3[k][0], b = T3[k][1], g = T3[k][2];
    const double H3 = c[a] * c[b] * c[g] - CS2 * (c[a] * kd(b, g) + c[b] * kd(a, g) + c[g] * kd(a, b));
    const T Tabg = q.S[a][b] * q.u[g] + q.S[a][g] * q.u[b] + q.S[b][g] * q.u[a] - T(2.0) * q.u[a] * q.u[b] * q.u[g];
    const bool xyz = (k == 6);
    const double coef = (xyz && !literal_xyz) ? 1.0 / (CS2 * CS2 * CS2) : 1.0 / (2.0 * CS2 * CS2 * CS2);
    third = third + T(coef * H3) * Tabg;
  }
  return q.rho * T(LAT.w[i]) * (T(1.0) + first + second + third);
}

// Moments of 27 distributions, Eq. (rho_u_stress): rho = sum f,
// rho u = sum c f + F/2, rho S = sum (c c - cs^2 delta) f.
template <class T>
void project(const T f[27], const double F[3], T m[10]) {
  for (int k = 0; k < 10; ++k) m[k] = T(0.0);
  for (int i = 0; i < 27; ++i) {
    const double* c = LAT.cd[i];
    m[0] = m[0] + f[i];
    for (int a = 0; a < 3; ++a) m[1 + a] = m[1 + a] + T(c[a]) * f[i];
    for (int p = 0; p < 6; ++p) m[4 + p] = m[4 + p] + T(c[PA[p]] * c[PB[p]] - CS2 * kd(PA[p], PB[p])) * f[i];
  }
  for (int a = 0; a < 3; ++a) m[1 + a] = m[1 + a] + T(0.5 * F[a]);
}

// Moment-space collision, App. A (the starred quantities are the inputs).
template <class T>
Cell<T> collide(const Cell<T>& s, const double F[3], double tau) {
  Cell<T> o;
  const T& rho = s.rho;
  const T Fv[3] = {T(F[0]), T(F[1]), T(F[2])};
  o.rho = rho;
  for (int a = 0; a < 3; ++a) o.u[a] = s.u[a] + Fv[a] / (T(2.0) * rho);
  // off-diagonal entries
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      o.S[a][b] = T(1.0 - 1.0 / tau) * s.S[a][b] + s.u[a] * s.u[b] / T(tau) +
                  T(2.0 * tau - 1.0) / (T(2.0 * tau) * rho) * (Fv[a] * s.u[b] + Fv[b] * s.u[a]);
    }
  // diagonal entries: alpha, with beta and gamma the two other axes
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, g = (a + 2) % 3;
    o.S[a][a] = T((tau - 1.0) / (3.0 * tau)) * (T(2.0) * s.S[a][a] - s.S[b][b] - s.S[g][g]) +
                (s.u[a] * s.u[a] + s.u[b] * s.u[b] + s.u[g] * s.u[g]) / T(3.0) +
                (T(2.0) * s.u[a] * s.u[a] - s.u[b] * s.u[b] - s.u[g] * s.u[g]) / T(3.0 * tau) +
                Fv[a] * s.u[a] / rho +
                T(tau - 1.0) / (T(3.0 * tau) * rho) * (T(2.0) * Fv[a] * s.u[a] - Fv[b] * s.u[b] - Fv[g] * s.u[g]);
  }
  return o;
}

// Stored moments (rho, rho u, rho S) -> paper variables (rho, u, S).
template <class T>
Cell<T> to_cell(const T m[10]) {
  Cell<T> q;
  q.rho = m[0];
  for (int a = 0; a < 3; ++a) q.u[a] = m[1 + a] / q.rho;
  for (int p = 0; p < 6; ++p) {
    q.S[PA[p]][PB[p]] = m[4 + p] / q.rho;
    q.S[PB[p]][PA[p]] = q.S[PA[p]][PB[p]];
  }
  return q;
}

}  // namespace

extern "C" {

// Grid and physics parameters.  Cell (x, y, z) has linear index
// x + nx * (y + ny * z); a field is 10 planes of nx*ny*nz values in the
// stored-moment order above.
struct OrcParams {
  int nx, ny, nz;
  int inflow;       // 1: x = 0 inflow face, x = nx-1 outflow face; 0: x periodic
  int literal_xyz;  // reading R1 switch
  double tau;
  double F[3];      // uniform body force
  double u_in[3];   // inflow velocity
  int wall_rule;    // 0: halfway bounce-back (R10); 1: moment wall at the link
                    // midpoint (R16); 2: moment wall where the link meets the
                    // obstacle meshes (R26)
  const double* objects;  // 256 x 9: center C, velocity V, angular velocity W of
                          // object id (mask value); NULL: all at rest at 0
  const float* tris;      // wall rule 2: ntris triangles, 9 floats each (x0 y0 z0 x1 ... z2)
  int64_t ntris;
  const uint8_t* tri_obj; // object id of each triangle
};

}  // extern "C"

namespace {

inline int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Triangles that may meet a link of each lattice point (wall rule 2): a
// link from x has length at most sqrt(3) and stays within one cell of x on
// every axis, so only triangles whose bounding box, widened by one cell,
// holds x can meet it.  Looking only at these gives the same nearest hit as
// testing every triangle.
struct MeshIndex {
  std::unordered_map<int64_t, std::vector<int64_t>> near;
  void build(const OrcParams& P) {
    for (int64_t k = 0; k < P.ntris; ++k) {
      const float* t = P.tris + 9 * k;
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        const double mn = std::min({double(t[a]), double(t[3 + a]), double(t[6 + a])});
        const double mx = std::max({double(t[a]), double(t[3 + a]), double(t[6 + a])});
        lo[a] = int(std::floor(mn)) - 1;
        hi[a] = int(std::ceil(mx)) + 1;
      }
      for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
          for (int x = lo[0]; x <= hi[0]; ++x) {
            if (x < 0 || y < 0 || z < 0 || x >= P.nx || y >= P.ny || z >= P.nz) continue;
            near[int64_t(x) + int64_t(P.nx) * (int64_t(y) + int64_t(P.ny) * z)].push_back(k);
          }
    }
  }
};

template <class T>
struct Grid {
  const OrcParams& P;
  const uint8_t* mask;
  int64_t N;
  MeshIndex mesh;
  Grid(const OrcParams& p, const uint8_t* m) : P(p), mask(m) {
    N = int64_t(p.nx) * p.ny * p.nz;
    if (p.wall_rule == 2 && p.tris) mesh.build(p);
  }
  int64_t idx(int x, int y, int z) const { return int64_t(x) + int64_t(P.nx) * (int64_t(y) + int64_t(P.ny) * z); }
  bool solid(int64_t c) const { return mask && mask[c]; }
};

// Where the segment from the origin to d meets triangle (v0, v1, v2) (all in
// coordinates relative to the segment's start): the parameter t in [0, 1] of
// the point t d, or -1 when it misses.  Points on an edge count as hits.
// Moller & Trumbore, "Fast, minimum storage ray-triangle intersection",
// J. Graphics Tools 2(1), 1997, restricted to the segment.
double segment_triangle(const double d[3], const double v0[3], const double v1[3], const double v2[3]) {
  const double tol = 1e-9;
  double e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = v1[a] - v0[a];
    e2[a] = v2[a] - v0[a];
  }
  const double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
  const double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
  if (std::fabs(det) < 1e-300) return -1.0;  // segment parallel to the triangle's plane
  const double inv = 1.0 / det;
  const double s[3] = {-v0[0], -v0[1], -v0[2]};
  const double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
  if (u < -tol || u > 1.0 + tol) return -1.0;
  const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
  const double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
  if (v < -tol || u + v > 1.0 + tol) return -1.0;
  const double t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
  if (t < -tol || t > 1.0 + tol) return -1.0;
  return std::min(std::max(t, 0.0), 1.0);
}

template <class T>
Cell<T> load_post(const OrcParams& P, const T* in, int64_t N, int64_t c) {
  T m[10];
  for (int k = 0; k < 10; ++k) m[k] = in[k * N + c];
  return collide(to_cell(m), P.F, P.tau);
}

// Velocity of object `id` at the midpoint p of the link from (x, y, z) along
// -c (R16): V + W x (p - C).
inline void wall_velocity_at(const OrcParams& P, int id, const double p[3], double u[3]) {
  double C[3] = {0, 0, 0}, V[3] = {0, 0, 0}, W[3] = {0, 0, 0};
  if (P.objects) {
    for (int a = 0; a < 3; ++a) {
      C[a] = P.objects[9 * id + a];
      V[a] = P.objects[9 * id + 3 + a];
      W[a] = P.objects[9 * id + 6 + a];
    }
  }
  const double r[3] = {p[0] - C[0], p[1] - C[1], p[2] - C[2]};
  u[0] = V[0] + W[1] * r[2] - W[2] * r[1];
  u[1] = V[1] + W[2] * r[0] - W[0] * r[2];
  u[2] = V[2] + W[0] * r[1] - W[1] * r[0];
}

inline void wall_velocity(const OrcParams& P, int id, int x, int y, int z, int cx, int cy, int cz, double u[3]) {
  const double p[3] = {x - 0.5 * cx, y - 0.5 * cy, z - 0.5 * cz};
  wall_velocity_at(P, id, p, u);
}

// The boundary point of the link from fluid cell (x, y, z) along -c to its
// solid source s (R16, R26): wall rule 2 takes the nearest point where the
// link meets a triangle (ties to the lowest triangle index) and that
// triangle's object; a link that meets no triangle, and wall rule 1, take the
// link midpoint and the object of s.  Returns whether a triangle was met.
template <class T>
bool link_boundary_point(const Grid<T>& G, int x, int y, int z, int cx, int cy, int cz, int64_t s, double p[3],
                         int* id) {
  const OrcParams& P = G.P;
  p[0] = x - 0.5 * cx;
  p[1] = y - 0.5 * cy;
  p[2] = z - 0.5 * cz;
  *id = G.mask[s];
  if (P.wall_rule != 2) return false;
  const auto it = G.mesh.near.find(G.idx(x, y, z));
  if (it == G.mesh.near.end()) return false;
  const double d[3] = {-double(cx), -double(cy), -double(cz)};
  double best = 2.0;
  int64_t bk = -1;
  for (const int64_t k : it->second) {
    const float* t = P.tris + 9 * k;
    const double v0[3] = {t[0] - double(x), t[1] - double(y), t[2] - double(z)};
    const double v1[3] = {t[3] - double(x), t[4] - double(y), t[5] - double(z)};
    const double v2[3] = {t[6] - double(x), t[7] - double(y), t[8] - double(z)};
    const double h = segment_triangle(d, v0, v1, v2);
    if (h >= 0.0 && (h < best || (h == best && k < bk))) {
      best = h;
      bk = k;
    }
  }
  if (bk < 0) return false;
  p[0] = x - best * cx;
  p[1] = y - best * cy;
  p[2] = z - best * cz;
  *id = P.tri_obj[bk];
  return true;
}

// f_i arriving at fluid cell (x, y, z) after the pull-stream, with the face
// and wall rules (R10, R11, R16).  post(c) returns the post-collision Cell of c.
template <class T, class PostFn>
T pulled(const Grid<T>& G, int x, int y, int z, int i, PostFn&& post) {
  const OrcParams& P = G.P;
  const int cx = LAT.c[i][0], cy = LAT.c[i][1], cz = LAT.c[i][2];
  const bool lit = P.literal_xyz != 0;
  if (P.inflow && x == 0 && cx == +1) {
    // moment boundary at the inflow face: rho^p = rho^x, u^p = u_in,
    // S^p = u^p u^p + (S^x - u^x u^x)
    const Cell<T> q = post(G.idx(x, y, z));
    Cell<T> p;
    p.rho = q.rho;
    for (int a = 0; a < 3; ++a) p.u[a] = T(P.u_in[a]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) p.S[a][b] = T(P.u_in[a] * P.u_in[b]) + (q.S[a][b] - q.u[a] * q.u[b]);
    return hermite_f(i, p, lit);
  }
  if (P.inflow && x == P.nx - 1 && cx == -1) {
    const int sy = wrap(y - cy, P.ny), sz = wrap(z - cz, P.nz);
    return hermite_f(i, post(G.idx(P.nx - 1, sy, sz)), lit);
  }
  int sx = x - cx;
  if (!P.inflow) sx = wrap(sx, P.nx);
  const int sy = wrap(y - cy, P.ny), sz = wrap(z - cz, P.nz);
  const int64_t s = G.idx(sx, sy, sz);
  if (G.solid(s)) {
    if (P.wall_rule == 0) return hermite_f(LAT.opp[i], post(G.idx(x, y, z)), lit);
    // moment wall (R16, R26): rho^p = rho^x, u^p of the object at p, S^p = u^p u^p + (S^x - u^x u^x)
    const Cell<T> q = post(G.idx(x, y, z));
    double pp[3], up[3];
    int id = 0;
    if (!link_boundary_point(G, x, y, z, cx, cy, cz, s, pp, &id) && P.wall_rule == 2) {
      // a link that meets no triangle is not coupled: the pull from the resting solid cell
      Cell<T> rest;
      rest.rho = T(1.0);
      for (int a = 0; a < 3; ++a) {
        rest.u[a] = T(0.0);
        for (int b = 0; b < 3; ++b) rest.S[a][b] = T(0.0);
      }
      return hermite_f(i, rest, lit);
    }
    wall_velocity_at(P, id, pp, up);
    Cell<T> pc;
    pc.rho = q.rho;
    for (int a = 0; a < 3; ++a) pc.u[a] = T(up[a]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) pc.S[a][b] = T(up[a] * up[b]) + (q.S[a][b] - q.u[a] * q.u[b]);
    return hermite_f(i, pc, lit);
  }
  return hermite_f(i, post(s), lit);
}

template <class T, class PostFn>
void new_moments(const Grid<T>& G, int x, int y, int z, PostFn&& post, T m[10]) {
  const int64_t c = G.idx(x, y, z);
  if (G.solid(c)) {
    for (int k = 0; k < 10; ++k) m[k] = T(0.0);
    m[0] = T(1.0);
    return;
  }
  T f[27];
  for (int i = 0; i < 27; ++i) f[i] = pulled(G, x, y, z, i, post);
  project(f, G.P.F, m);
}

template <class T>
void step_grid(const OrcParams& P, const uint8_t* mask, const T* in, T* out, int nthreads) {
  Grid<T> G(P, mask);
  const int64_t N = G.N;
  std::vector<Cell<T>> post(N);
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int z = 0; z < P.nz; ++z)
    for (int y = 0; y < P.ny; ++y)
      for (int x = 0; x < P.nx; ++x) {
        const int64_t c = G.idx(x, y, z);
        if (!G.solid(c)) post[c] = load_post(P, in, N, c);
      }
  auto get = [&](int64_t c) -> const Cell<T>& { return post[c]; };
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int z = 0; z < P.nz; ++z)
    for (int y = 0; y < P.ny; ++y)
      for (int x = 0; x < P.nx; ++x) {
        T m[10];
        new_moments(G, x, y, z, get, m);
        const int64_t c = G.idx(x, y, z);
        for (int k = 0; k < 10; ++k) out[k * N + c] = m[k];
      }
}

// ---------------------------------------------------------------------------
// 16-bit codec, Sec. 5.3.
// ---------------------------------------------------------------------------

// Stored codec variables: rho, u (3), N = rho S - rho u u (6), readings R2, R3.
const double Q_LO[10] = {0.8, -0.4, -0.4, -0.4, -0.1, -0.1, -0.1, -0.1, -0.1, -0.1};
const double Q_HI[10] = {1.5, 0.4, 0.4, 0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
const uint32_t QMAX = 65535u;  // 2^b - 1 with b = 16

// pcg_hash: one LCG step followed by the RXS-M-XS output permutation
// (Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 9(3), 2020).
uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// Per-step key.  mode 1: a new key every step; mode 2: one static pattern.
uint32_t dither_key(uint32_t t, uint32_t seed, int mode) {
  const uint32_t tt = (mode == 2) ? 0u : t;
  return pcg_hash(seed ^ pcg_hash(tt));
}

// Ten dither values for cell idx at step t (reading R6).
void dither(uint32_t idx, uint32_t t, uint32_t seed, int mode, double xi[10], uint32_t h[2]) {
  if (mode == 0) {
    for (int k = 0; k < 10; ++k) xi[k] = 0.0;
    h[0] = h[1] = 0u;
    return;
  }
  const uint32_t key = dither_key(t, seed, mode);
  const uint32_t h1 = pcg_hash(idx ^ key);
  const uint32_t h2 = pcg_hash(h1 ^ 0x9E3779B9u);
  h[0] = h1;
  h[1] = h2;
  for (int k = 0; k < 10; ++k) {
    const uint32_t src = (k < 5) ? h1 : h2;
    const uint32_t v = (src >> (6 * (k % 5))) & 63u;
    xi[k] = (double(v) + 0.5) / 64.0 - 0.5;
  }
}

// q = floor(m' (2^b - 1) + 1/2 + xi), m' = (m - min)/(max - min), taken in
// double precision exactly as Sec. 5.3 writes it (half-way values go up), and
// saturated (R5).
uint16_t encode_one(double m, int k, double xi) {
  const double mp = (m - Q_LO[k]) / (Q_HI[k] - Q_LO[k]);
  const double v = std::floor(mp * double(QMAX) + 0.5 + xi);
  if (!(v >= 0.0)) return 0;  // also maps NaN to 0
  if (v >= double(QMAX)) return uint16_t(QMAX);
  return uint16_t(v);
}

double decode_one(uint32_t q, int k) { return Q_LO[k] + double(q) * ((Q_HI[k] - Q_LO[k]) / double(QMAX)); }

// Stored moments (rho, j, P) -> codec variables (rho, u, N).
void moments_to_codec_vars(const double m[10], double v[10]) {
  const double rho = m[0];
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = m[1 + a] / rho;
  v[0] = rho;
  for (int a = 0; a < 3; ++a) v[1 + a] = u[a];
  for (int p = 0; p < 6; ++p) v[4 + p] = m[4 + p] - rho * u[PA[p]] * u[PB[p]];
}

void codec_vars_to_moments(const double v[10], double m[10]) {
  const double rho = v[0];
  m[0] = rho;
  for (int a = 0; a < 3; ++a) m[1 + a] = rho * v[1 + a];
  for (int p = 0; p < 6; ++p) m[4 + p] = v[4 + p] + rho * v[1 + PA[p]] * v[1 + PB[p]];
}

// Five words per cell, two codes per word, low half first:
// w0 = rho|ux, w1 = uy|uz, w2 = Nxx|Nyy, w3 = Nzz|Nxy, w4 = Nxz|Nyz.
void pack(const uint16_t q[10], uint32_t w[5]) {
  for (int p = 0; p < 5; ++p) w[p] = uint32_t(q[2 * p]) | (uint32_t(q[2 * p + 1]) << 16);
}
void unpack(const uint32_t w[5], uint32_t q[10]) {
  for (int p = 0; p < 5; ++p) {
    q[2 * p] = w[p] & 0xFFFFu;
    q[2 * p + 1] = w[p] >> 16;
  }
}

void encode_cell(const double m[10], uint32_t idx, uint32_t t, uint32_t seed, int mode, uint32_t w[5]) {
  double v[10], xi[10];
  uint32_t h[2];
  moments_to_codec_vars(m, v);
  dither(idx, t, seed, mode, xi, h);
  uint16_t q[10];
  for (int k = 0; k < 10; ++k) q[k] = encode_one(v[k], k, xi[k]);
  pack(q, w);
}

void decode_cell(const uint32_t w[5], double m[10]) {
  uint32_t q[10];
  unpack(w, q);
  double v[10];
  for (int k = 0; k < 10; ++k) v[k] = decode_one(q[k], k);
  codec_vars_to_moments(v, m);
}

// ---- b_rho_u / b_S bit allocation (the study of the double-layer vortex,
// Sec. 6): b1 bits for rho and u, b2 bits for N, the same ranges, rounding
// and dither, and the ten codes concatenated low bit first into
// ceil((4 b1 + 6 b2) / 32) words (R18).  16/16 is the layout above.
struct Bits {
  int b1, b2;
  int of(int k) const { return k < 4 ? b1 : b2; }
  int words() const { return (4 * b1 + 6 * b2 + 31) / 32; }
};

uint32_t encode_one_b(double m, int k, double xi, int b) {
  const uint32_t qmax = (1u << b) - 1u;
  const double mp = (m - Q_LO[k]) / (Q_HI[k] - Q_LO[k]);
  const double v = std::floor(mp * double(qmax) + 0.5 + xi);
  if (!(v >= 0.0)) return 0;
  if (v >= double(qmax)) return qmax;
  return uint32_t(v);
}

double decode_one_b(uint32_t q, int k, int b) {
  return Q_LO[k] + double(q) * ((Q_HI[k] - Q_LO[k]) / double((1u << b) - 1u));
}

// Stream bit o of a cell is bit o % 32 of its word o / 32; code k occupies
// stream bits [o_k, o_k + b_k), o_k the sum of the widths before it.
void pack_bits(const uint32_t q[10], const Bits& B, uint32_t* w) {
  for (int i = 0; i < B.words(); ++i) w[i] = 0u;
  int o = 0;
  for (int k = 0; k < 10; ++k) {
    for (int t = 0; t < B.of(k); ++t) w[(o + t) / 32] |= ((q[k] >> t) & 1u) << ((o + t) % 32);
    o += B.of(k);
  }
}

void unpack_bits(const uint32_t* w, const Bits& B, uint32_t q[10]) {
  int o = 0;
  for (int k = 0; k < 10; ++k) {
    q[k] = 0u;
    for (int t = 0; t < B.of(k); ++t) q[k] |= ((w[(o + t) / 32] >> ((o + t) % 32)) & 1u) << t;
    o += B.of(k);
  }
}

void encode_cell_b(const double m[10], uint32_t idx, uint32_t t, uint32_t seed, int mode, const Bits& B,
                   uint32_t* w) {
  double v[10], xi[10];
  uint32_t h[2];
  moments_to_codec_vars(m, v);
  dither(idx, t, seed, mode, xi, h);
  uint32_t q[10];
  for (int k = 0; k < 10; ++k) q[k] = encode_one_b(v[k], k, xi[k], B.of(k));
  pack_bits(q, B, w);
}

void decode_cell_b(const uint32_t* w, const Bits& B, double m[10]) {
  uint32_t q[10];
  unpack_bits(w, B, q);
  double v[10];
  for (int k = 0; k < 10; ++k) v[k] = decode_one_b(q[k], k, B.of(k));
  codec_vars_to_moments(v, m);
}

// ---------------------------------------------------------------------------
// Adjoint of one step, lam_prev = J(m_t)^T lam_next.  The per-cell Jacobians
// of f+ (and of the inflow distributions) are taken by complex step of the
// functions above, so the adjoint is the exact transpose of this oracle's own
// step, assembled link by link in the same pull order.
// ---------------------------------------------------------------------------

using cd = std::complex<double>;
constexpr double CS_H = 1e-30;

}  // namespace

extern "C" {

int orc_version() { return 1; }

void orc_lattice(int* c, double* w, int* opp) {
  for (int i = 0; i < 27; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = LAT.c[i][a];
    w[i] = LAT.w[i];
    opp[i] = LAT.opp[i];
  }
}

// h(rho, u, S) for one cell; S6 in the order xx, yy, zz, xy, xz, yz.
void orc_reconstruct(double rho, const double* u, const double* S6, int literal_xyz, double* f27) {
  Cell<double> q;
  q.rho = rho;
  for (int a = 0; a < 3; ++a) q.u[a] = u[a];
  for (int p = 0; p < 6; ++p) q.S[PA[p]][PB[p]] = q.S[PB[p]][PA[p]] = S6[p];
  for (int i = 0; i < 27; ++i) f27[i] = hermite_f(i, q, literal_xyz != 0);
}

void orc_project(const double* f27, const double* F, double* m10) {
  const double zero[3] = {0, 0, 0};
  project(f27, F ? F : zero, m10);
}

void orc_collide(double rho, const double* u, const double* S6, const double* F, double tau, double* out10) {
  Cell<double> s;
  s.rho = rho;
  for (int a = 0; a < 3; ++a) s.u[a] = u[a];
  for (int p = 0; p < 6; ++p) s.S[PA[p]][PB[p]] = s.S[PB[p]][PA[p]] = S6[p];
  const double zero[3] = {0, 0, 0};
  const Cell<double> o = collide(s, F ? F : zero, tau);
  out10[0] = o.rho;
  for (int a = 0; a < 3; ++a) out10[1 + a] = o.u[a];
  for (int p = 0; p < 6; ++p) out10[4 + p] = o.S[PA[p]][PB[p]];
}

// f+ = h(collide(m)) for one cell given stored moments m10, complex input
// (pass im = NULL for a real evaluation).
void orc_post_collision_f(const OrcParams* P, const double* m_re, const double* m_im, double* f_re, double* f_im) {
  cd m[10];
  for (int k = 0; k < 10; ++k) m[k] = cd(m_re[k], m_im ? m_im[k] : 0.0);
  const Cell<cd> q = collide(to_cell(m), P->F, P->tau);
  for (int i = 0; i < 27; ++i) {
    const cd f = hermite_f(i, q, P->literal_xyz != 0);
    f_re[i] = f.real();
    if (f_im) f_im[i] = f.imag();
  }
}

int orc_step(const OrcParams* P, const uint8_t* mask, const double* in, double* out, int nthreads) {
  step_grid<double>(*P, mask, in, out, nthreads > 0 ? nthreads : 1);
  return 0;
}

// ---- The paper's mixed-precision pipeline (Sec. 5.3, atomic accumulation):
// the 16-bit buffer holds post-collision moments; a step streams them into
// FP32 post-stream moments (the boundary rules applied), then collides and
// re-encodes them.  Without quantization, stream(collide(m)) is the step of m.

// Post-stream moments of every cell from post-collision moments m_post
// (rho, rho u+, rho S+ per cell); solid cells get rest.
int orc_stream_post(const OrcParams* P, const uint8_t* mask, const double* m_post, double* m_ps, int nthreads) {
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  std::vector<Cell<double>> post(N);
  for (int64_t c = 0; c < N; ++c) {
    double m[10];
    for (int k = 0; k < 10; ++k) m[k] = m_post[k * N + c];
    post[c] = to_cell(m);
  }
  auto get = [&](int64_t c) -> const Cell<double>& { return post[c]; };
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        double m[10];
        new_moments(G, x, y, z, get, m);
        const int64_t c = G.idx(x, y, z);
        for (int k = 0; k < 10; ++k) m_ps[k * N + c] = m[k];
      }
  return 0;
}

// Post-collision moments (rho, rho u+, rho S+) of every cell (App. A); solid
// cells get rest.
int orc_collide_field(const OrcParams* P, const uint8_t* mask, const double* m_ps, double* m_post) {
  const int64_t N = int64_t(P->nx) * P->ny * P->nz;
  for (int64_t c = 0; c < N; ++c) {
    double out[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!(mask && mask[c])) {
      double m[10];
      for (int k = 0; k < 10; ++k) m[k] = m_ps[k * N + c];
      const Cell<double> q = collide(to_cell(m), P->F, P->tau);
      out[0] = q.rho;
      for (int a = 0; a < 3; ++a) out[1 + a] = q.rho * q.u[a];
      for (int p = 0; p < 6; ++p) out[4 + p] = q.rho * q.S[PA[p]][PB[p]];
    }
    for (int k = 0; k < 10; ++k) m_post[k * N + c] = out[k];
  }
  return 0;
}

void orc_q16_encode(const double* m, const uint8_t* mask, int64_t N, uint32_t t, uint32_t seed, int mode,
                    uint32_t* w);
void orc_q16_decode(const uint32_t* w, int64_t N, double* m);

// One step of the mixed pipeline on 16-bit post-collision codes: decode,
// stream (m_ps receives the FP64 post-stream moments), collide, encode with
// the dither of step t.
int orc_mixed_q16_step(const OrcParams* P, const uint8_t* mask, const uint32_t* in, uint32_t* out, double* m_ps,
                       uint32_t t, uint32_t seed, int mode, int nthreads) {
  const int64_t N = int64_t(P->nx) * P->ny * P->nz;
  std::vector<double> post(10 * N), post2(10 * N);
  orc_q16_decode(in, N, post.data());
  orc_stream_post(P, mask, post.data(), m_ps, nthreads);
  orc_collide_field(P, mask, m_ps, post2.data());
  orc_q16_encode(post2.data(), mask, N, t, seed, mode, out);
  return 0;
}

// Force and torque on every object during the step from `in` (R17), summed
// over the links of the fluid cells whose source is solid: out[6 id + 0..2]
// force, out[6 id + 3..5] torque about the object's center, ids 0..255.
int orc_object_forces(const OrcParams* P, const uint8_t* mask, const double* in, double* out) {
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  for (int k = 0; k < 256 * 6; ++k) out[k] = 0.0;
  if (!mask) return 0;
  auto get = [&](int64_t c) { return load_post(*P, in, N, c); };
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        const int64_t c = G.idx(x, y, z);
        if (G.solid(c)) continue;
        for (int i = 0; i < 27; ++i) {
          const int cx = LAT.c[i][0], cy = LAT.c[i][1], cz = LAT.c[i][2];
          if (P->inflow && ((x == 0 && cx == +1) || (x == P->nx - 1 && cx == -1))) continue;
          int sx = x - cx;
          if (!P->inflow) sx = wrap(sx, P->nx);
          const int64_t s = G.idx(sx, wrap(y - cy, P->ny), wrap(z - cz, P->nz));
          if (!G.solid(s)) continue;
          double pp[3];
          int id = 0;
          link_boundary_point(G, x, y, z, cx, cy, cz, s, pp, &id);
          const double f_in = pulled(G, x, y, z, i, get);
          const double f_out = hermite_f(LAT.opp[i], get(c), P->literal_xyz != 0);
          double dp[3];
          for (int a = 0; a < 3; ++a) dp[a] = -(f_in + f_out) * LAT.cd[i][a];
          double C[3] = {0, 0, 0};
          if (P->objects)
            for (int a = 0; a < 3; ++a) C[a] = P->objects[9 * id + a];
          const double r[3] = {pp[0] - C[0], pp[1] - C[1], pp[2] - C[2]};
          double* o = out + 6 * id;
          for (int a = 0; a < 3; ++a) o[a] += dp[a];
          o[3] += r[1] * dp[2] - r[2] * dp[1];
          o[4] += r[2] * dp[0] - r[0] * dp[2];
          o[5] += r[0] * dp[1] - r[1] * dp[0];
        }
      }
  return 0;
}

// The boundary points of wall rule 2 (R26): for every link from a fluid cell
// to a solid source (with the x faces open, not the face links), writes
// (cell, i, met a triangle, p_x, p_y, p_z, object id) into out (7 doubles per
// link, up to cap links); returns the number of links.
int64_t orc_mesh_links(const OrcParams* P, const uint8_t* mask, double* out, int64_t cap) {
  Grid<double> G(*P, mask);
  int64_t n = 0;
  if (!mask) return 0;
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        const int64_t c = G.idx(x, y, z);
        if (G.solid(c)) continue;
        for (int i = 0; i < 27; ++i) {
          const int cx = LAT.c[i][0], cy = LAT.c[i][1], cz = LAT.c[i][2];
          if (P->inflow && ((x == 0 && cx == +1) || (x == P->nx - 1 && cx == -1))) continue;
          int sx = x - cx;
          if (!P->inflow) sx = wrap(sx, P->nx);
          const int64_t s = G.idx(sx, wrap(y - cy, P->ny), wrap(z - cz, P->nz));
          if (!G.solid(s)) continue;
          double pp[3];
          int id = 0;
          const bool met = link_boundary_point(G, x, y, z, cx, cy, cz, s, pp, &id);
          if (n < cap) {
            double* o = out + 7 * n;
            o[0] = double(c);
            o[1] = i;
            o[2] = met ? 1.0 : 0.0;
            o[3] = pp[0];
            o[4] = pp[1];
            o[5] = pp[2];
            o[6] = id;
          }
          ++n;
        }
      }
  return n;
}

int orc_step_f32(const OrcParams* P, const uint8_t* mask, const float* in, float* out, int nthreads) {
  step_grid<float>(*P, mask, in, out, nthreads > 0 ? nthreads : 1);
  return 0;
}

// One step in complex arithmetic (complex-step derivatives of the step).
int orc_step_cs(const OrcParams* P, const uint8_t* mask, const double* in_re, const double* in_im, double* out_re,
                double* out_im, int nthreads) {
  const int64_t n = int64_t(P->nx) * P->ny * P->nz * 10;
  std::vector<cd> in(n), out(n);
  for (int64_t k = 0; k < n; ++k) in[k] = cd(in_re[k], in_im[k]);
  step_grid<cd>(*P, mask, in.data(), out.data(), nthreads > 0 ? nthreads : 1);
  for (int64_t k = 0; k < n; ++k) {
    out_re[k] = out[k].real();
    out_im[k] = out[k].imag();
  }
  return 0;
}

// New moments at a list of cells only (for sampled comparisons at full size).
int orc_step_cells(const OrcParams* P, const uint8_t* mask, const double* in, int64_t ncells, const int64_t* cells,
                   double* out, int nthreads) {
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  auto get = [&](int64_t c) { return load_post(*P, in, N, c); };
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t k = 0; k < ncells; ++k) {
    const int64_t c = cells[k];
    const int x = int(c % P->nx), y = int((c / P->nx) % P->ny), z = int(c / (int64_t(P->nx) * P->ny));
    new_moments(G, x, y, z, get, out + 10 * k);
  }
  return 0;
}

uint32_t orc_pcg_hash(uint32_t v) { return pcg_hash(v); }

void orc_dither(uint32_t idx, uint32_t t, uint32_t seed, int mode, double* xi10, uint32_t* h2) {
  uint32_t h[2];
  dither(idx, t, seed, mode, xi10, h);
  if (h2) {
    h2[0] = h[0];
    h2[1] = h[1];
  }
}

uint32_t orc_encode_one(double m, int k, double xi) { return encode_one(m, k, xi); }
uint32_t orc_encode_one_b(double m, int k, double xi, int b) { return encode_one_b(m, k, xi, b); }
double orc_decode_one(uint32_t q, int k) { return decode_one(q, k); }

// Encode a field of stored moments (10 planes) into 5 planes of words.
// Solid cells get the rest state without dither.
void orc_q16_encode(const double* m, const uint8_t* mask, int64_t N, uint32_t t, uint32_t seed, int mode,
                    uint32_t* w) {
  for (int64_t c = 0; c < N; ++c) {
    double mc[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool sol = mask && mask[c];
    if (!sol)
      for (int k = 0; k < 10; ++k) mc[k] = m[k * N + c];
    uint32_t wc[5];
    encode_cell(mc, uint32_t(c), t, seed, sol ? 0 : mode, wc);
    for (int p = 0; p < 5; ++p) w[p * N + c] = wc[p];
  }
}

void orc_q16_decode(const uint32_t* w, int64_t N, double* m) {
  for (int64_t c = 0; c < N; ++c) {
    uint32_t wc[5];
    for (int p = 0; p < 5; ++p) wc[p] = w[p * N + c];
    double mc[10];
    decode_cell(wc, mc);
    for (int k = 0; k < 10; ++k) m[k * N + c] = mc[k];
  }
}

// Packed codes with b1 / b2 bits (R18): words() planes of N words.
int orc_qb_encode(const double* m, const uint8_t* mask, int64_t N, uint32_t t, uint32_t seed, int mode, int b1, int b2,
                  uint32_t* w) {
  const Bits B{b1, b2};
  if (b1 < 2 || b1 > 16 || b2 < 2 || b2 > 16) return -1;
  for (int64_t c = 0; c < N; ++c) {
    double mc[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool sol = mask && mask[c];
    if (!sol)
      for (int k = 0; k < 10; ++k) mc[k] = m[k * N + c];
    uint32_t wc[5];
    encode_cell_b(mc, uint32_t(c), t, seed, sol ? 0 : mode, B, wc);
    for (int p = 0; p < B.words(); ++p) w[p * N + c] = wc[p];
  }
  return 0;
}

int orc_qb_decode(const uint32_t* w, int64_t N, int b1, int b2, double* m) {
  const Bits B{b1, b2};
  if (b1 < 2 || b1 > 16 || b2 < 2 || b2 > 16) return -1;
  for (int64_t c = 0; c < N; ++c) {
    uint32_t wc[5];
    for (int p = 0; p < B.words(); ++p) wc[p] = w[p * N + c];
    double mc[10];
    decode_cell_b(wc, B, mc);
    for (int k = 0; k < 10; ++k) m[k * N + c] = mc[k];
  }
  return 0;
}

// Codes <-> packed words only (for pins of the layout): q is 10 x N.
int orc_qb_pack(const uint32_t* q, int64_t N, int b1, int b2, uint32_t* w) {
  const Bits B{b1, b2};
  for (int64_t c = 0; c < N; ++c) {
    uint32_t qc[10], wc[5];
    for (int k = 0; k < 10; ++k) qc[k] = q[k * N + c];
    pack_bits(qc, B, wc);
    for (int p = 0; p < B.words(); ++p) w[p * N + c] = wc[p];
  }
  return 0;
}

int orc_qb_step(const OrcParams* P, const uint8_t* mask, const uint32_t* in, uint32_t* out, uint32_t t, uint32_t seed,
                int mode, int b1, int b2, int nthreads) {
  const int64_t N = int64_t(P->nx) * P->ny * P->nz;
  std::vector<double> m(10 * N), m2(10 * N);
  if (orc_qb_decode(in, N, b1, b2, m.data()) != 0) return -1;
  step_grid<double>(*P, mask, m.data(), m2.data(), nthreads > 0 ? nthreads : 1);
  return orc_qb_encode(m2.data(), mask, N, t, seed, mode, b1, b2, out);
}

// One 16-bit step: decode -> FP64 step -> encode with the dither of step t.
int orc_q16_step(const OrcParams* P, const uint8_t* mask, const uint32_t* in, uint32_t* out, uint32_t t, uint32_t seed,
                 int mode, int nthreads) {
  const int64_t N = int64_t(P->nx) * P->ny * P->nz;
  std::vector<double> m(10 * N), m2(10 * N);
  orc_q16_decode(in, N, m.data());
  step_grid<double>(*P, mask, m.data(), m2.data(), nthreads > 0 ? nthreads : 1);
  orc_q16_encode(m2.data(), mask, N, t, seed, mode, out);
  return 0;
}

// 16-bit step at a list of cells only; out holds 5 words per listed cell.
int orc_q16_step_cells(const OrcParams* P, const uint8_t* mask, const uint32_t* in, uint32_t t, uint32_t seed, int mode,
                       int64_t ncells, const int64_t* cells, uint32_t* out, int nthreads) {
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  auto get = [&](int64_t c) {
    uint32_t wc[5];
    for (int p = 0; p < 5; ++p) wc[p] = in[p * N + c];
    double mc[10];
    decode_cell(wc, mc);
    return collide(to_cell(mc), P->F, P->tau);
  };
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t k = 0; k < ncells; ++k) {
    const int64_t c = cells[k];
    const int x = int(c % P->nx), y = int((c / P->nx) % P->ny), z = int(c / (int64_t(P->nx) * P->ny));
    double mc[10];
    new_moments(G, x, y, z, get, mc);
    const bool sol = G.solid(c);
    encode_cell(mc, uint32_t(c), t, seed, sol ? 0 : mode, out + 5 * k);
  }
  return 0;
}

// lam_prev = J(m_t)^T lam_next for one FP64 step (fields of 10 planes).
int orc_adjoint_step(const OrcParams* P, const uint8_t* mask, const double* m_t, const double* lam_next,
                     double* lam_prev, int nthreads) {
  if (P->wall_rule != 0) return -1;  // the adjoint follows bounce-back walls only
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  const bool lit = P->literal_xyz != 0;
  // Jf[c][i][k] = d f+_i(c) / d m_k(c), one cell at a time (cells in parallel)
  std::vector<double> Jf(size_t(N) * 270, 0.0);
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t c = 0; c < N; ++c) {
    if (G.solid(c)) continue;
    for (int k = 0; k < 10; ++k) {
      cd m[10];
      for (int q = 0; q < 10; ++q) m[q] = cd(m_t[q * N + c], q == k ? CS_H : 0.0);
      const Cell<cd> post = collide(to_cell(m), P->F, P->tau);
      for (int i = 0; i < 27; ++i) Jf[size_t(c) * 270 + i * 10 + k] = hermite_f(i, post, lit).imag() / CS_H;
    }
  }
  for (int64_t q = 0; q < 10 * N; ++q) lam_prev[q] = 0.0;
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        const int64_t c = G.idx(x, y, z);
        if (G.solid(c)) continue;
        for (int i = 0; i < 27; ++i) {
          const double* cv = LAT.cd[i];
          // d(new moments at c) / d f_i(c)
          double phi[10];
          phi[0] = 1.0;
          for (int a = 0; a < 3; ++a) phi[1 + a] = cv[a];
          for (int p = 0; p < 6; ++p) phi[4 + p] = cv[PA[p]] * cv[PB[p]] - CS2 * kd(PA[p], PB[p]);
          double lf = 0.0;
          for (int k = 0; k < 10; ++k) lf += phi[k] * lam_next[k * N + c];
          const int cx = LAT.c[i][0], cy = LAT.c[i][1], cz = LAT.c[i][2];
          if (P->inflow && x == 0 && cx == +1) {
            // inflow distribution depends on the post-collision moments of c itself
            for (int k = 0; k < 10; ++k) {
              cd m[10];
              for (int q = 0; q < 10; ++q) m[q] = cd(m_t[q * N + c], q == k ? CS_H : 0.0);
              const Cell<cd> qq = collide(to_cell(m), P->F, P->tau);
              Cell<cd> p;
              p.rho = qq.rho;
              for (int a = 0; a < 3; ++a) p.u[a] = cd(P->u_in[a], 0.0);
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) p.S[a][b] = cd(P->u_in[a] * P->u_in[b]) + (qq.S[a][b] - qq.u[a] * qq.u[b]);
              lam_prev[k * N + c] += lf * hermite_f(i, p, lit).imag() / CS_H;
            }
            continue;
          }
          int64_t src;
          int dir = i;
          if (P->inflow && x == P->nx - 1 && cx == -1) {
            src = G.idx(P->nx - 1, wrap(y - cy, P->ny), wrap(z - cz, P->nz));
          } else {
            int sx = x - cx;
            if (!P->inflow) sx = wrap(sx, P->nx);
            src = G.idx(sx, wrap(y - cy, P->ny), wrap(z - cz, P->nz));
            if (G.solid(src)) {
              src = c;
              dir = LAT.opp[i];
            }
          }
          const double* J = &Jf[size_t(src) * 270 + dir * 10];
          for (int k = 0; k < 10; ++k) lam_prev[k * N + src] += lf * J[k];
        }
      }
  return 0;
}

// lam_prev at chosen cells only: the same transpose as orc_adjoint_step,
// gathered per source cell s instead of scattered per output cell.  f+_i(s)
// reaches the new moments of (a) c = s + c_i by pull streaming (c fluid, x
// inside the domain when the x faces are open), (b) with open faces and s on
// the outflow face x = nx - 1, the face cell (nx - 1, y + c_iy, z + c_iz) for
// c_ix = -1 (zero gradient), (c) s itself on a bounce-back link: f_opp(i)(s)
// = f+_i(s) when s + c_i is solid; and (d) on the inflow face x = 0 the
// inflow distributions of s depend on the post-collision moments of s.
// Solid cells get zeros.  out: ncells x 10.
int orc_adjoint_step_cells(const OrcParams* P, const uint8_t* mask, const double* m_t, const double* lam_next,
                           int64_t ncells, const int64_t* cells, double* out, int nthreads) {
  if (P->wall_rule != 0) return -1;
  Grid<double> G(*P, mask);
  const int64_t N = G.N;
  const bool lit = P->literal_xyz != 0;
  auto phi_of = [](int i, double phi[10]) {
    const double* cv = LAT.cd[i];
    phi[0] = 1.0;
    for (int a = 0; a < 3; ++a) phi[1 + a] = cv[a];
    for (int p = 0; p < 6; ++p) phi[4 + p] = cv[PA[p]] * cv[PB[p]] - CS2 * kd(PA[p], PB[p]);
  };
  auto lam_dot = [&](int i, int64_t c) {
    double phi[10];
    phi_of(i, phi);
    double lf = 0.0;
    for (int k = 0; k < 10; ++k) lf += phi[k] * lam_next[k * N + c];
    return lf;
  };
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t n = 0; n < ncells; ++n) {
    const int64_t s = cells[n];
    double* o = out + 10 * n;
    for (int k = 0; k < 10; ++k) o[k] = 0.0;
    if (G.solid(s)) continue;
    const int x = int(s % P->nx), y = int((s / P->nx) % P->ny), z = int(s / (int64_t(P->nx) * P->ny));
    // J[i][k] = d f+_i(s) / d m_k(s)
    double J[27][10];
    for (int k = 0; k < 10; ++k) {
      cd m[10];
      for (int q = 0; q < 10; ++q) m[q] = cd(m_t[q * N + s], q == k ? CS_H : 0.0);
      const Cell<cd> post = collide(to_cell(m), P->F, P->tau);
      for (int i = 0; i < 27; ++i) J[i][k] = hermite_f(i, post, lit).imag() / CS_H;
    }
    for (int i = 0; i < 27; ++i) {
      const int cx = LAT.c[i][0], cy = LAT.c[i][1], cz = LAT.c[i][2];
      double lf = 0.0;
      // (a) pull streaming into c = s + c_i
      int tx = x + cx;
      bool inside = true;
      if (P->inflow) inside = tx >= 0 && tx < P->nx;
      else tx = wrap(tx, P->nx);
      if (inside) {
        const int64_t c = G.idx(tx, wrap(y + cy, P->ny), wrap(z + cz, P->nz));
        if (!G.solid(c)) lf += lam_dot(i, c);
        // (c) bounce-back: s + c_i solid sends f+_i(s) back into s as f_opp(i)(s)
        else lf += lam_dot(LAT.opp[i], s);
      }
      // (b) zero-gradient outflow: face cells take f+_i of their face neighbour
      if (P->inflow && x == P->nx - 1 && cx == -1) {
        const int64_t c = G.idx(P->nx - 1, wrap(y + cy, P->ny), wrap(z + cz, P->nz));
        if (!G.solid(c)) lf += lam_dot(i, c);
      }
      if (lf != 0.0)
        for (int k = 0; k < 10; ++k) o[k] += lf * J[i][k];
    }
    // (d) the inflow distributions of s (c_ix = +1 on x = 0)
    if (P->inflow && x == 0) {
      for (int i = 0; i < 27; ++i) {
        if (LAT.c[i][0] != +1) continue;
        const double lf = lam_dot(i, s);
        for (int k = 0; k < 10; ++k) {
          cd m[10];
          for (int q = 0; q < 10; ++q) m[q] = cd(m_t[q * N + s], q == k ? CS_H : 0.0);
          const Cell<cd> qq = collide(to_cell(m), P->F, P->tau);
          Cell<cd> pp;
          pp.rho = qq.rho;
          for (int a = 0; a < 3; ++a) pp.u[a] = cd(P->u_in[a], 0.0);
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) pp.S[a][b] = cd(P->u_in[a] * P->u_in[b]) + (qq.S[a][b] - qq.u[a] * qq.u[b]);
          o[k] += lf * hermite_f(i, pp, lit).imag() / CS_H;
        }
      }
    }
  }
  return 0;
}

}  // extern "C"
