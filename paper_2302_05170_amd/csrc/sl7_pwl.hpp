// Piecewise-linear compilation of ReLU collocation networks (host side).
#pragma once

#include <memory>
#include <mutex>
#include <vector>

#include "sl7_host.hpp"

namespace sl7 {

// The map Y -> (y_0..y_{m-1}) of one instance as P affine pieces in FP64:
// piece p covers [brk[p-1], brk[p]) (brk[-1] = -inf, brk[P-1] = +inf) and
// gives y_j = c[p m + j] + a[p m + j] (Y - o[p]).
// With theta derivatives (compile_pwl(..., with_theta = true)):
// dy_j/dtheta_k = da[(p n_theta + k) m + j] Y + db[(p n_theta + k) m + j]
// on piece p (the pieces' activation pattern held fixed, as back-propagation
// through the network holds its ReLU masks).
// Device layout of one instance's tables (see build_pwl_tables).
struct PwlBlob {
  std::vector<char> bytes;
  size_t rec = 0, brk = 0, grid = 0;
  int P = 0, cells = 0;
  double g0 = 0.0, ih = 0.0;
};

struct PwlPieces {
  int P = 0, m = 0, n_theta = 0;
  std::vector<double> brk, o, a, c, da, db;
  // serialized tables by [FP64][with theta], built on first use
  std::mutex mu;
  std::shared_ptr<const PwlBlob> blob[2][2];
};

int compile_pwl(const Mlp& H, const sl7_problem& pr, int max_pieces, PwlPieces& out,
                bool with_theta);
void grid_shape(const PwlPieces& pw, int& cells, double& g0, double& inv_h);

// Most pieces a compiled network may have.
constexpr int kPwlMaxPieces = 1 << 16;

// Compiles (or finds) the tables of n instances, uploads them into ws.pwl in
// the lane arithmetic's type and fills the instances' table fields.
// with_theta: records of kPwlAdjStride entries carrying the theta
// derivatives (the adjoint), else kPwlStride.
int build_pwl_tables(const sl7_problem* prs, int n, Mlp* H, bool f64, bool with_theta,
                     std::vector<InstDev>& inst, hipStream_t stream, Workspace& ws);

}  // namespace sl7
