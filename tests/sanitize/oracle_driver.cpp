// Driver for a sanitizer build of the oracle (address and undefined-behaviour
// checks on the host): every entry point of les_oracle.cpp runs once on small
// blocks that exercise periodic, superposed and Dirichlet directions and all
// face types.  The test that builds it checks only that the run is clean and
// that every result is finite.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/les_oracle.cpp"

static int bad = 0;
static void check_finite(const char* what, const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) {
      std::printf("non-finite %s[%zu]\n", what, i);
      ++bad;
      return;
    }
}

struct Block {
  orc_dims d;
  size_t N;
  std::vector<double> xyz, Q, m;
};

// Smooth wavy mapping (periodic up to a translation) and a smooth state.
static Block make_block(int ni, int nj, int nk, int b0, int b1, int b2) {
  Block B;
  B.d = orc_dims{};
  B.d.ni = ni; B.d.nj = nj; B.d.nk = nk;
  B.d.bc[0] = b0; B.d.bc[1] = b1; B.d.bc[2] = b2;
  B.N = orc_box_nodes(&B.d);
  const int pi = ni + 4, pj = nj + 4, pk = nk + 4;
  B.xyz.resize(3 * B.N);
  B.Q.resize(5 * B.N);
  B.m.resize(10 * B.N);
  const double pr[3] = {double(b0 == 2 ? ni - 1 : ni), double(b1 == 2 ? nj - 1 : nj), double(b2 == 2 ? nk - 1 : nk)};
  for (int k = 0; k < pk; ++k)
    for (int j = 0; j < pj; ++j)
      for (int i = 0; i < pi; ++i) {
        const size_t n = ((size_t)k * pj + j) * pi + i;
        const double I = i - 2, J = j - 2, K = k - 2;
        const double a = 2 * M_PI * I / pr[0], b = 2 * M_PI * J / pr[1], c = 2 * M_PI * K / pr[2];
        const double W = 0.15 * std::sin(a) * std::sin(b) * std::sin(c);
        B.xyz[n] = (I + W) / pr[0];
        B.xyz[B.N + n] = (J + 0.5 * W) / pr[1];
        B.xyz[2 * B.N + n] = (K - 0.3 * W) / pr[2];
        const double rho = 1.0 + 0.05 * std::cos(a + b), u = 0.3 + 0.05 * std::sin(b + c), v = -0.1 + 0.05 * std::cos(c);
        const double w = 0.05 * std::sin(a), p = (1.0 + 0.03 * std::sin(a + c)) / 1.4;
        B.Q[n] = rho;
        B.Q[B.N + n] = rho * u;
        B.Q[2 * B.N + n] = rho * v;
        B.Q[3 * B.N + n] = rho * w;
        B.Q[4 * B.N + n] = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w);
      }
  orc_metrics(&B.d, B.xyz.data(), B.m.data());
  return B;
}

int main() {
  orc_params P{1.4, 0.72, 0.9, 3e-3, 1.0, 0.383, 1.0 / 1.4, 1, 0.17, 0.25, 1.0 / 64, 0.5, 0.5};
  std::printf("threads %d\n", orc_threads(2));
  const int bcs[4][3] = {{0, 0, 0}, {2, 0, 1}, {1, 1, 0}, {0, 1, 2}};
  for (int t = 0; t < 4; ++t) {
    Block B = make_block(9, 8, 7, bcs[t][0], bcs[t][1], bcs[t][2]);
    if (t == 2) {  // faces on the Dirichlet directions i and j: entrance, exit, far field
      B.d.face[0] = 1; B.d.face[1] = 2; B.d.face[2] = 3; B.d.face[3] = 3;
      B.d.p_exit[1] = 1.0 / 1.4;
      B.d.outside = B.Q.data();
    }
    const size_t N = B.N;
    std::vector<double> R(5 * N), dR(5 * N), dQ(5 * N, 1e-3), f(5 * 7 * 8, 1e-4), df(5 * 7 * 8, 1.0);
    orc_residual(&B.d, &P, B.m.data(), B.Q.data(), f.data(), 3, R.data());
    check_finite("R", R.data(), R.size());
    orc_residual_tangent(&B.d, &P, B.m.data(), B.Q.data(), dQ.data(), f.data(), df.data(), 3, R.data(), dR.data());
    check_finite("dR", dR.data(), dR.size());
    double dt = orc_cfl_dt(&B.d, &P, B.m.data(), B.Q.data());
    std::vector<double> Q(B.Q), stages(25 * N), norms(10);
    double used = orc_rk_step(&B.d, &P, B.m.data(), Q.data(), 0.0, f.data(), 3, norms.data(), stages.data());
    check_finite("norms", norms.data(), 10);
    if (!(used > 0.0) || used != dt) ++bad;
    std::vector<double> Qt(B.Q), dQt(dQ);
    orc_rk_step_tangent(&B.d, &P, B.m.data(), Qt.data(), dQt.data(), dt, f.data(), df.data(), 3);
    check_finite("dQ", dQt.data(), dQt.size());
    std::vector<double> Qo(B.Q);
    double dJ = 0.0;
    double J = orc_objective_rollout(&B.d, &P, B.m.data(), Qo.data(), nullptr, f.data(), df.data(), 3, 5, 1.0 / 1.4,
                                     2, dt, &dJ);
    std::vector<double> Qo2(B.Q);
    double J2 = orc_objective(&B.d, &P, B.m.data(), Qo2.data(), f.data(), 3, 5, 1.0 / 1.4, 2, dt);
    if (!std::isfinite(J) || !std::isfinite(dJ) || J != J2) ++bad;
    std::vector<double> acc(12 * 8 * 9, 0.0);
    orc_stats(&B.d, &P, B.Q.data(), acc.data());
    check_finite("stats", acc.data(), acc.size());
    std::vector<double> g(B.Q);
    if (t != 2) orc_fill_ghosts(&B.d, g.data(), 5);  // faces need the metrics: the next call
    orc_fill_ghosts_faces(&B.d, &P, B.m.data(), g.data());
    check_finite("ghosts", g.data(), g.size());
  }
  double yr = 1.0, yi = 0.0;
  orc_rk_scalar(-1.0, 0.5, 0.1, &yr, &yi);
  std::printf("%s\n", bad ? "FAILED" : "clean");
  return bad ? 1 : 0;
}
