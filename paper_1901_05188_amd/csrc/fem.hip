// Element integrals, material tensors and gather-form assembly on the GPU.
//
// Section 2 of the paper: strain eq-strain, Hooke's law eq-hooke with an
// orthotropic ply rotated by a standard tensor rotation, weak form eq-fe and
// the element-wise Gauss-integrated assembly eqn:fe_matrix_system; Section 6
// eq-fe-darcy for the scalar problem.  Q1 hexahedra, 2x2x2 Gauss points.
//
// The rotated stiffness is built with the 6x6 Bond transformation
// C' = M C M^T (Voigt order 11,22,33,23,13,12, engineering shear), with the
// orthotropic normal block inverted in closed form by cofactors.
#include "gn_internal.h"

namespace {

struct Geo {
  const double* xn0;
  const double* xn1;
  const double* xn2;
  int map_kind;
  double mx0, mx1, mtan;
};

__device__ inline double ramp(const Geo& g, double x) {
  if (g.map_kind != 1) return 0.0;
  double c = x < g.mx0 ? g.mx0 : (x > g.mx1 ? g.mx1 : x);
  return g.mtan * (c - g.mx0);
}

// node coordinates of element (ex,ey,ez), local node a = ax + 2ay + 4az
__device__ inline void elem_coords(const Geo& g, int ex, int ey, int ez, double X[8][3]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    double x = g.xn0[ex + ax];
    X[a][0] = x;
    X[a][1] = g.xn1[ey + ay];
    X[a][2] = g.xn2[ez + az] + ramp(g, x);
  }
}

// shape-function gradients in physical space and det J at reference point q
__device__ inline double grad_at(const double X[8][3], double xi, double eta, double zeta,
                                 double G[8][3], double N[8]) {
  double dN[8][3];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    double sx = (a & 1) ? 1.0 : -1.0, sy = ((a >> 1) & 1) ? 1.0 : -1.0,
           sz = ((a >> 2) & 1) ? 1.0 : -1.0;
    double fx = 0.5 * (1.0 + sx * xi), fy = 0.5 * (1.0 + sy * eta), fz = 0.5 * (1.0 + sz * zeta);
    N[a] = fx * fy * fz;
    dN[a][0] = 0.5 * sx * fy * fz;
    dN[a][1] = 0.5 * sy * fx * fz;
    dN[a][2] = 0.5 * sz * fx * fy;
  }
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // J[d][k] = dx_d/dxi_k
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[d][k] += X[a][d] * dN[a][k];
  double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  double inv = 1.0 / det;
  // K = J^-1 : K[k][d] = dxi_k/dx_d
  double K[3][3];
  K[0][0] = c00 * inv;
  K[1][0] = c01 * inv;
  K[2][0] = c02 * inv;
  K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
  K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
  K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
  K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
  K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
  K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      G[a][d] = dN[a][0] * K[0][d] + dN[a][1] * K[1][d] + dN[a][2] * K[2][d];
  return det;
}

// rotated orthotropic stiffness (Voigt, engineering shear)
__device__ void material_stiffness(const double* c9, double theta, double tilt, double C[6][6]) {
  double E1 = c9[0], E2 = c9[1], E3 = c9[2], G12 = c9[3], G13 = c9[4], G23 = c9[5];
  double n12 = c9[6], n13 = c9[7], n23 = c9[8];
  // normal compliance block and its cofactor inverse
  double s[3][3] = {{1.0 / E1, -n12 / E1, -n13 / E1},
                    {-n12 / E1, 1.0 / E2, -n23 / E2},
                    {-n13 / E1, -n23 / E2, 1.0 / E3}};
  double cf[3][3];
  cf[0][0] = s[1][1] * s[2][2] - s[1][2] * s[2][1];
  cf[0][1] = s[1][2] * s[2][0] - s[1][0] * s[2][2];
  cf[0][2] = s[1][0] * s[2][1] - s[1][1] * s[2][0];
  cf[1][1] = s[0][0] * s[2][2] - s[0][2] * s[2][0];
  cf[1][2] = s[0][1] * s[2][0] - s[0][0] * s[2][1];
  cf[2][2] = s[0][0] * s[1][1] - s[0][1] * s[1][0];
  double det = s[0][0] * cf[0][0] + s[0][1] * cf[0][1] + s[0][2] * cf[0][2];
  double C0[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C0[i][j] = 0.0;
  C0[0][0] = cf[0][0] / det;
  C0[1][1] = cf[1][1] / det;
  C0[2][2] = cf[2][2] / det;
  C0[0][1] = C0[1][0] = cf[0][1] / det;
  C0[0][2] = C0[2][0] = cf[0][2] / det;
  C0[1][2] = C0[2][1] = cf[1][2] / det;
  C0[3][3] = G23;
  C0[4][4] = G13;
  C0[5][5] = G12;
  // rotation: Q = Ry(tilt) Rz(theta); material axes -> global axes
  double c = cos(theta), sn = sin(theta), ct = cos(tilt), st = sin(tilt);
  double Rz[3][3] = {{c, -sn, 0.0}, {sn, c, 0.0}, {0.0, 0.0, 1.0}};
  double Ry[3][3] = {{ct, 0.0, -st}, {0.0, 1.0, 0.0}, {st, 0.0, ct}};
  double a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      a[i][j] = Ry[i][0] * Rz[0][j] + Ry[i][1] * Rz[1][j] + Ry[i][2] * Rz[2][j];
  // Bond stress transformation
  const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
  double M[6][6];
  for (int I = 0; I < 6; ++I) {
    int i = vi[I], j = vj[I];
    for (int J = 0; J < 6; ++J) {
      int p = vi[J], q = vj[J];
      M[I][J] = (p == q) ? a[i][p] * a[j][p] : a[i][p] * a[j][q] + a[i][q] * a[j][p];
    }
  }
  double T[6][6];
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double acc = 0.0;
      for (int K = 0; K < 6; ++K) acc += M[I][K] * C0[K][J];
      T[I][J] = acc;
    }
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double acc = 0.0;
      for (int K = 0; K < 6; ++K) acc += T[I][K] * M[J][K];
      C[I][J] = acc;
    }
}

__global__ void k_material(int n_elem, const double* mats, const int* emat, const double* eang,
                           const double* etilt, double* Cout) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  double C[6][6];
  material_stiffness(mats + 9 * emat[e], eang ? eang[e] : 0.0, etilt ? etilt[e] : 0.0, C);
  double* o = Cout + (int64_t)e * 36;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) o[i * 6 + j] = 0.5 * (C[i][j] + C[j][i]);
}

// one thread per (element, row i) of the 24x24 element stiffness.  Row i =
// 3 a_i + c_i of B^T C B det J w needs only the three rows of C that meet the
// nonzero strain entries of column i of B: (c_i, 4 or 3, 5 or 4), scaled by the
// gradient components (x,z,y), (y,z,x) or (z,y,x) of node a_i.  Every private
// array is indexed by compile-time constants (the node a_i and component c_i
// are picked by selects), so nothing spills to scratch memory.
__global__ __launch_bounds__(128) void k_ke_elastic(Geo g, int nex, int ney, int n_elem, const double* Cm,
                                                    double* Ke) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)n_elem * 24) return;
  int e = (int)(tid / 24), i = (int)(tid % 24);
  int ex = e % nex, ey = (e / nex) % ney, ez = e / (nex * ney);
  double X[8][3];
  elem_coords(g, ex, ey, ez, X);
  const int ai = i / 3, ci = i % 3;
  const int r1 = ci == 0 ? 4 : 3, r2 = ci == 2 ? 4 : 5;
  const double* cp = Cm + (int64_t)e * 36;
  double crow[3][6];
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    crow[0][b] = cp[ci * 6 + b];
    crow[1][b] = cp[r1 * 6 + b];
    crow[2][b] = cp[r2 * 6 + b];
  }
  double acc[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) acc[k] = 0.0;
  const double gp = 0.57735026918962576451;  // 1/sqrt(3)
  for (int q = 0; q < 8; ++q) {
    double G[8][3], N[8];
    double det = grad_at(X, (q & 1) ? gp : -gp, ((q >> 1) & 1) ? gp : -gp,
                         ((q >> 2) & 1) ? gp : -gp, G, N);
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      gx = a == ai ? G[a][0] : gx;
      gy = a == ai ? G[a][1] : gy;
      gz = a == ai ? G[a][2] : gz;
    }
    const double g0 = ci == 0 ? gx : (ci == 1 ? gy : gz);
    const double g1 = ci == 2 ? gy : gz;
    const double g2 = ci == 0 ? gy : gx;
    double v[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) v[b] = (g0 * crow[0][b] + g1 * crow[1][b] + g2 * crow[2][b]) * det;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      double hx = G[a][0], hy = G[a][1], hz = G[a][2];
      acc[3 * a + 0] += v[0] * hx + v[4] * hz + v[5] * hy;
      acc[3 * a + 1] += v[1] * hy + v[3] * hz + v[5] * hx;
      acc[3 * a + 2] += v[2] * hz + v[3] * hy + v[4] * hx;
    }
  }
  double* o = Ke + (int64_t)e * 576 + i * 24;
#pragma unroll
  for (int k = 0; k < 24; ++k) o[k] = acc[k];
}

__global__ __launch_bounds__(128) void k_ke_scalar(Geo g, int nex, int ney, int n_elem, const double* kel,
                                                   double* Ke) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)n_elem * 8) return;
  int e = (int)(tid / 8), i = (int)(tid % 8);
  int ex = e % nex, ey = (e / nex) % ney, ez = e / (nex * ney);
  double X[8][3];
  elem_coords(g, ex, ey, ez, X);
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  const double gp = 0.57735026918962576451;
  for (int q = 0; q < 8; ++q) {
    double G[8][3], N[8];
    double det = grad_at(X, (q & 1) ? gp : -gp, ((q >> 1) & 1) ? gp : -gp,
                         ((q >> 2) & 1) ? gp : -gp, G, N);
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      gx = a == i ? G[a][0] : gx;
      gy = a == i ? G[a][1] : gy;
      gz = a == i ? G[a][2] : gz;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += (gx * G[k][0] + gy * G[k][1] + gz * G[k][2]) * det;
  }
  double ke = kel[e];
  double* o = Ke + (int64_t)e * 64 + i * 8;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = ke * acc[k];
}

// gather-form assembly: one thread per (node, neighbour offset d, row comp c)
template <int NC>
__global__ void k_assemble(int nex, int ney, int nez, const double* Ke, const uint8_t* dir,
                           double* A) {
  const int NX = nex + 1, NY = ney + 1, NZ = nez + 1;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n_node * 27 * NC) return;
  int64_t node = tid % n_node;
  int dc = (int)(tid / n_node);
  int d = dc / NC, c = dc % NC;
  int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
  int i = (int)(node % NX), j = (int)((node / NX) % NY), k = (int)(node / ((int64_t)NX * NY));
  int i2 = i + dx, j2 = j + dy, k2 = k + dz;
  double val[NC];
#pragma unroll
  for (int c2 = 0; c2 < NC; ++c2) val[c2] = 0.0;
  bool inside = i2 >= 0 && i2 < NX && j2 >= 0 && j2 < NY && k2 >= 0 && k2 < NZ;
  if (inside) {
    int exl = max(max(i, i2) - 1, 0), exh = min(min(i, i2), nex - 1);
    int eyl = max(max(j, j2) - 1, 0), eyh = min(min(j, j2), ney - 1);
    int ezl = max(max(k, k2) - 1, 0), ezh = min(min(k, k2), nez - 1);
    for (int ez = ezl; ez <= ezh; ++ez)
      for (int ey = eyl; ey <= eyh; ++ey)
        for (int ex = exl; ex <= exh; ++ex) {
          int64_t e = ex + (int64_t)nex * (ey + (int64_t)ney * ez);
          int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
          int a2 = (i2 - ex) + 2 * (j2 - ey) + 4 * (k2 - ez);
          const double* row = Ke + e * (64 * NC * NC) + (int64_t)(a * NC + c) * (8 * NC);
#pragma unroll
          for (int c2 = 0; c2 < NC; ++c2) val[c2] += row[a2 * NC + c2];
        }
    int64_t nb = i2 + (int64_t)NX * (j2 + (int64_t)NY * k2);
    bool dr = dir[node * NC + c];
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) {
      bool dcol = dir[nb * NC + c2];
      if (dr || dcol) val[c2] = (d == 13 && c2 == c) ? 1.0 : 0.0;
    }
  }
#pragma unroll
  for (int c2 = 0; c2 < NC; ++c2) A[((int64_t)(d * NC + c) * NC + c2) * n_node + node] = val[c2];
}

// load vector: one thread per node; body force + top-face traction, all rhs
template <int NC>
__global__ void k_load(Geo g, int nex, int ney, int nez, int nrhs, const double* body,
                       const double* trac, const uint8_t* dir, double* b) {
  const int NX = nex + 1, NY = ney + 1, NZ = nez + 1;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n_node) return;
  int i = (int)(node % NX), j = (int)((node / NX) % NY), k = (int)(node / ((int64_t)NX * NY));
  double acc[NC][4];
  const int RB = 4;  // rhs handled per pass
  const double gp = 0.57735026918962576451;
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    for (int c = 0; c < NC; ++c)
      for (int r = 0; r < RB; ++r) acc[c][r] = 0.0;
    for (int ez = max(k - 1, 0); ez <= min(k, nez - 1); ++ez)
      for (int ey = max(j - 1, 0); ey <= min(j, ney - 1); ++ey)
        for (int ex = max(i - 1, 0); ex <= min(i, nex - 1); ++ex) {
          int64_t e = ex + (int64_t)nex * (ey + (int64_t)ney * ez);
          int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
          double X[8][3];
          bool need_body = false;
          if (body) {
            for (int c = 0; c < NC; ++c) need_body |= body[e * NC + c] != 0.0;
          }
          bool top = trac && ez == nez - 1 && (a >> 2) == 1;
          if (!need_body && !top) continue;
          elem_coords(g, ex, ey, ez, X);
          if (need_body) {
            double s = 0.0;
            for (int q = 0; q < 8; ++q) {
              double G[8][3], N[8];
              double det = grad_at(X, (q & 1) ? gp : -gp, ((q >> 1) & 1) ? gp : -gp,
                                   ((q >> 2) & 1) ? gp : -gp, G, N);
              s += N[a] * det;
            }
            for (int c = 0; c < NC; ++c)
              for (int r = 0; r < RB && r0 + r < nrhs; ++r) acc[c][r] += body[e * NC + c] * s;
          }
          if (top) {
            double s = 0.0;
            for (int q = 0; q < 4; ++q) {
              double G[8][3], N[8];
              double xi = (q & 1) ? gp : -gp, eta = (q & 2) ? gp : -gp;
              grad_at(X, xi, eta, 1.0, G, N);
              // tangents dx/dxi, dx/deta on the face zeta = 1
              double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
              for (int b2 = 4; b2 < 8; ++b2) {
                double sx = (b2 & 1) ? 1.0 : -1.0, sy = ((b2 >> 1) & 1) ? 1.0 : -1.0;
                double d1 = 0.25 * sx * (1.0 + sy * eta), d2 = 0.25 * sy * (1.0 + sx * xi);
                for (int d = 0; d < 3; ++d) {
                  t1[d] += X[b2][d] * d1;
                  t2[d] += X[b2][d] * d2;
                }
              }
              double nx = t1[1] * t2[2] - t1[2] * t2[1];
              double ny = t1[2] * t2[0] - t1[0] * t2[2];
              double nz = t1[0] * t2[1] - t1[1] * t2[0];
              s += N[a] * sqrt(nx * nx + ny * ny + nz * nz);
            }
            int64_t face = ex + (int64_t)nex * ey;
            for (int r = 0; r < RB && r0 + r < nrhs; ++r)
              for (int c = 0; c < NC; ++c)
                acc[c][r] += trac[((int64_t)(r0 + r) * nex * ney + face) * NC + c] * s;
          }
        }
    for (int r = 0; r < RB && r0 + r < nrhs; ++r)
      for (int c = 0; c < NC; ++c) {
        int64_t dof = node * NC + c;
        b[(int64_t)(r0 + r) * n_node * NC + dof] = dir[dof] ? 0.0 : acc[c][r];
      }
  }
}

Geo make_geo(const gn_problem* p) {
  Geo g;
  g.xn0 = p->d_xn[0];
  g.xn1 = p->d_xn[1];
  g.xn2 = p->d_xn[2];
  g.map_kind = p->map_kind;
  g.mx0 = p->map_par[0];
  g.mx1 = p->map_par[1];
  g.mtan = tan(p->map_par[2]);
  return g;
}

}  // namespace

namespace gnk {

void element_matrices(gn_problem* p, const double* d_mats, int n_mat, const int* d_emat,
                      const double* d_eang, const double* d_etilt, const double* d_ek,
                      hipStream_t s) {
  (void)n_mat;
  Geo g = make_geo(p);
  int n_elem = (int)p->n_elem;
  if (p->pde == 1) {
    double* dC = (double*)gnh::dev_alloc(sizeof(double) * 36 * (size_t)n_elem);
    hipLaunchKernelGGL(k_material, dim3((n_elem + 127) / 128), dim3(128), 0, s, n_elem, d_mats,
                       d_emat, d_eang, d_etilt, dC);
    GN_CHECK_LAUNCH();
    int64_t nt = (int64_t)n_elem * 24;
    hipLaunchKernelGGL(k_ke_elastic, dim3((unsigned)((nt + 127) / 128)), dim3(128), 0, s, g,
                       p->ne[0], p->ne[1], n_elem, dC, p->d_Ke);
    GN_CHECK_LAUNCH();
    GN_HIP(hipStreamSynchronize(s));
    gnh::dev_free(dC);
  } else {
    int64_t nt = (int64_t)n_elem * 8;
    hipLaunchKernelGGL(k_ke_scalar, dim3((unsigned)((nt + 127) / 128)), dim3(128), 0, s, g,
                       p->ne[0], p->ne[1], n_elem, d_ek, p->d_Ke);
    GN_CHECK_LAUNCH();
  }
}

void assemble_matrix(gn_problem* p, hipStream_t s) {
  int64_t nt = p->n_node * 27 * p->nc;
  dim3 grid((unsigned)((nt + 255) / 256));
  if (p->nc == 3)
    hipLaunchKernelGGL(k_assemble<3>, grid, dim3(256), 0, s, p->ne[0], p->ne[1], p->ne[2],
                       p->d_Ke, p->d_dir, p->d_A);
  else
    hipLaunchKernelGGL(k_assemble<1>, grid, dim3(256), 0, s, p->ne[0], p->ne[1], p->ne[2],
                       p->d_Ke, p->d_dir, p->d_A);
  GN_CHECK_LAUNCH();
}

void assemble_load(const gn_problem* p, const double* d_body, const double* d_trac, int nrhs, double* d_out,
                   hipStream_t s) {
  Geo g = make_geo(p);
  dim3 grid((unsigned)((p->n_node + 127) / 128));
  if (p->nc == 3)
    hipLaunchKernelGGL(k_load<3>, grid, dim3(128), 0, s, g, p->ne[0], p->ne[1], p->ne[2],
                       nrhs, d_body, d_trac, p->d_dir, d_out);
  else
    hipLaunchKernelGGL(k_load<1>, grid, dim3(128), 0, s, g, p->ne[0], p->ne[1], p->ne[2],
                       nrhs, d_body, d_trac, p->d_dir, d_out);
  GN_CHECK_LAUNCH();
}

}  // namespace gnk
