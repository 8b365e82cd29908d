// Runs the FP64 oracle on a small hand and grid without Python, so the
// oracle can be built with AddressSanitizer and UBSan.
#include <cmath>
#include <cstdio>
#include <vector>

#include "oracle_api.h"

int main() {
  // palm plus a 2-link finger; contacts on every link
  const int L = 3, nd = 6 + L - 1, Nc = 9;
  int parent[L] = {-1, 0, 1};
  double origin[L * 12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0,
                           1, 0, 0, 0.01, 0, 1, 0, 0, 0, 0, 1, 0.02,
                           0, -1, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0.03};
  double axis[L * 3] = {0, 0, 1, 0, 1, 0, 1, 0, 0};
  double lo[nd] = {0}, up[nd] = {0};
  for (int j = 6; j < nd; ++j) { lo[j] = -0.5; up[j] = 1.5; }
  double cl[Nc * 3];
  int lk[Nc];
  for (int i = 0; i < Nc; ++i) {
    lk[i] = i % L;
    cl[3 * i] = 0.004 * i; cl[3 * i + 1] = -0.003 * (i % 2); cl[3 * i + 2] = 0.002 * (i % 3);
  }
  ohand h{L, parent, origin, axis, lo, up, Nc, cl, lk};
  const int n = 12;
  std::vector<float> vals(n * n * n);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double x = -0.05 + 0.01 * i, y = -0.05 + 0.01 * j, z = -0.05 + 0.01 * k;
        vals[(k * n + j) * n + i] = static_cast<float>(std::sqrt(x * x + y * y + z * z) - 0.03);
      }
  oobject o{};
  o.kind = OBJ_GRID;
  o.n = n;
  o.lo[0] = o.lo[1] = o.lo[2] = -0.05;
  o.h = 0.01;
  o.values = vals.data();
  oparams p{1e-3, 1.0, 3, 1.0, 0.002, 0.1, 1.0, 1e4, 1e-2, 1.0, 1e-12};
  const int B = 3;
  double q[B * nd] = {0};
  for (int b = 0; b < B; ++b) {
    q[b * nd + 0] = 0.01 * b - 0.01; q[b * nd + 2] = 0.02; q[b * nd + 3] = 0.3 * b;
    for (int j = 6; j < nd; ++j) q[b * nd + j] = 0.2 * j - 1.0 + 0.1 * b;
  }
  double loss[B], terms[4 * B], grad[B * nd], margins[3 * B], fd[B * nd];
  int ex[B * nd];
  if (oracle_step(&h, &o, &p, B, q, loss, terms, grad, margins, 2)) return 1;
  if (oracle_fd_grad(&h, &o, &p, B, q, 1e-6, fd, ex, 2)) return 2;
  std::vector<double> poses(7 * (p.K + 1) * 6), samples(7 * p.K * Nc * 6), pw(Nc * 3);
  if (oracle_trace(&h, &o, &p, q, poses.data(), samples.data(), pw.data())) return 3;
  double qq[B * nd], m[B * nd] = {0}, v[B * nd] = {0}, fl[B], ft[4 * B];
  int rank[B];
  for (int i = 0; i < B * nd; ++i) qq[i] = q[i];
  if (oracle_optimize(&h, &o, &p, B, qq, 3, 0.01, 1e-3, 0.9, 0.999, 1e-8, 0, fl, ft, rank, nullptr, 2)) return 4;
  for (int b = 0; b < B; ++b)
    if (!std::isfinite(loss[b]) || !std::isfinite(fl[b])) return 5;
  // the literal Gauss-Seidel sweep
  oparams pg = p;
  pg.projection = 1;
  double lgs[B], ggs[B * nd];
  if (oracle_step(&h, &o, &pg, B, q, lgs, nullptr, ggs, nullptr, 2)) return 6;
  // evaluation metrics of weighted samples, then the best two by loss
  double sa[Nc], sv[Nc];
  for (int i = 0; i < Nc; ++i) { sa[i] = 1e-5 * (i + 1); sv[i] = 1e-7 * (i + 1); }
  oeval ev{Nc, lk, cl, sa, Nc, lk, cl, sv};
  const double thr[3] = {0.002, 0.005, 0.009};
  double met[B * 4], slack[B * 4], mean[4];
  int top[2];
  if (oracle_evaluate(&h, &o, B, q, &ev, 3, thr, 1e-6, met, slack, 2)) return 7;
  if (oracle_select_top(B, loss, 0, 2, 4, met, top, mean)) return 8;
  // a tetrahedron mesh, flat and curved
  const double tv[12] = {0, 0, 0, 0.05, 0, 0, 0, 0.05, 0, 0, 0, 0.05};
  const int tf[12] = {0, 2, 1, 0, 1, 3, 0, 3, 2, 1, 2, 3};
  double tn[12];
  for (int i = 0; i < 4; ++i) {
    double c[3], len = 0.0;
    for (int k = 0; k < 3; ++k) { c[k] = tv[3 * i + k] - 0.0125; len += c[k] * c[k]; }
    for (int k = 0; k < 3; ++k) tn[3 * i + k] = c[k] / std::sqrt(len);
  }
  const double pts[9] = {0.01, 0.01, 0.01, 0.1, -0.02, 0.03, 0.02, 0.02, -0.01};
  double rho[3], grd[9], clo[9], dfl[3], gap[3], spr[3];
  int face[3];
  for (double alpha : {0.0, 0.75}) {
    omesh msh{4, tv, tn, 4, tf, alpha};
    if (oracle_mesh_sdf(&msh, 3, pts, rho, grd, clo, face, dfl, gap, spr)) return 9;
    if (!(rho[0] < 0.0) || !(rho[1] > 0.0)) return 10;
  }
  int top3[3];
  if (oracle_select_top(B, loss, 1, 3, 0, nullptr, top3, nullptr)) return 11;
  // the seven-query central-difference normal, in the step and the sampler
  oobject ofd = o;
  ofd.fd_normal = 1;
  double lfd[B], gfd[B * nd], sphi[3], sgrad[9], shess[27], smarg[3];
  if (oracle_step(&h, &ofd, &p, B, q, lfd, nullptr, gfd, nullptr, 2)) return 12;
  if (oracle_sample(&ofd, 3, pts, sphi, sgrad, shess, smarg)) return 13;
  std::printf("oracle ok %g %g %g\n", loss[0], loss[1], loss[2]);
  (void)m; (void)v;
  return 0;
}
