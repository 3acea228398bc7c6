// Host-side internals of the Seven-League library: error helpers, device
// buffers, per-device workspaces and the network handle.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sl7_internal.hpp"

namespace sl7 {

constexpr int kMaxGhNodes = 16;  // sl7_gh_nodes accepts m in [1, 16]

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int n_theta(int model);
int current_device(int* dev);
int gh_nodes(int m, double* x, double* w);

// A device allocation that only grows.  `generation` changes whenever the
// address changes (captured graphs keyed on it must be rebuilt).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  uint64_t generation = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  int reserve(size_t n);
};

// Pinned host staging for host-to-device uploads.  An upload enqueued from
// it may still be in flight when the call returns; the event recorded after
// it is waited on before the buffer is written again or freed.
struct Staging {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
  Staging() = default;
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  ~Staging();
  // waits for the previous upload, then makes room for n bytes
  int acquire(size_t n);
  // enqueues the upload of n bytes from offset off to dst on stream and
  // records the event (which then also covers earlier uploads from this
  // buffer on the same stream)
  int upload(void* dst, size_t off, size_t n, hipStream_t stream, const char* what);
};

// Scratch of one device, shared by the calls made on it (serialised by mu).
struct Workspace {
  std::mutex mu;
  int n_cu = 0;
  DevBuf inst, prefix, order, counter, partials, stats, chunks;
  DevBuf pwl;     // piecewise-linear tables of the instances (PWL modes)
  DevBuf cdc;     // per-step tables of the 7L-CDC variant
  Staging stage_inst, stage_pwl, stage_cdc;
  DevBuf aux[8];  // adjoint checkpoints, trainer buffers, ...
  sl7_stats* stats_host = nullptr;
  int stats_host_n = 0;
  int stats_host_reserve(int n);
  // end of the last call's work on the workspace, and the stream it ran on
  hipEvent_t done = nullptr;
  hipStream_t done_stream = nullptr;
};

Workspace& workspace(int dev);

// One call's hold on a device workspace: its lock for the call, and its
// buffers for the call's device work.  begin() makes the work enqueued on `s`
// wait for the previous call's (which may be on another stream); the
// destructor records the end of this call's work, so the next call waits for
// it in turn.  Calls that do not synchronise may thus be issued on any
// streams.
class WsLease {
 public:
  WsLease(Workspace& ws, hipStream_t s) : ws_(ws), s_(s), lk_(ws.mu) {}
  ~WsLease();
  WsLease(const WsLease&) = delete;
  WsLease& operator=(const WsLease&) = delete;
  int begin();

 private:
  Workspace& ws_;
  hipStream_t s_;
  std::lock_guard<std::mutex> lk_;
  bool begun_ = false;
};

struct PwlPieces;

// Next value of the process-wide network version counter.
uint64_t next_mlp_version();

// The network handle behind sl7_mlp.
struct Mlp {
  sl7_mlp_desc d;
  std::vector<float> params;
  std::vector<int64_t> W_off, b_off;
  std::string meta;
  std::mutex mu;
  int device = -1;
  std::unique_ptr<DevBuf> pack[6];  // MFMA register layouts, by precision
  std::unique_ptr<DevBuf> net64, w0full, w0n, c0n;
  // one-path-per-lane layouts (net_lane.hpp) in FP64 / FP32 and the theta
  // weights of the first layer (FP64) for the lane kernels and the adjoint
  std::unique_ptr<DevBuf> lane64, wth64;  // FP64 lane layout of the adjoint sweep
  std::unique_ptr<DevBuf> adj_img, adj_img_x3;  // LDS images of the MFMA adjoint sweep
  // compiled piecewise-linear forms by instance (model, dt, theta); cleared
  // with the device copies whenever the parameters change
  std::map<std::array<double, 5>, std::shared_ptr<PwlPieces>> pwl_cache;
  // unique in the process: a fresh value on creation and whenever the
  // parameters change, so (handle, version) never names two networks
  uint64_t version = next_mlp_version();

  void layout();
  float W(int l, int o, int k) const;
  float b(int l, int o) const;
  void drop_device();
  int ensure_device(int prec);
  int ensure_adjoint(int prec);
};

int64_t n_params_of(const sl7_mlp_desc& d);
// Builds and uploads H's FP64 lane layout (FP64 adjoint sweep and FP64
// simulation) and its theta weights; the caller holds H.mu.
int upload_lane_layout(const Mlp& H, std::unique_ptr<DevBuf>& net, std::unique_ptr<DevBuf>& wth);
int check_desc(const sl7_mlp_desc* d);
int check_problem(const sl7_problem* pr, const Mlp* H, int prec, const char* name);
int check_plan(const sl7_plan* p, int prec);
// The default launch plan for a launch of n_blocks 64-path blocks on n_cu
// compute units (n_blocks < 0: size not known).
int default_plan(int prec, int64_t n_blocks, int n_cu, sl7_plan* p);
int64_t total_blocks(const sl7_problem* prs, int n);
// pwl_theta: in the PWL modes, build the adjoint's records (with theta
// derivatives) instead of the simulation's.
int prepare_instances(const sl7_problem* prs, int n, const Mlp* H, int prec, uint64_t seed,
                      void* YT_dev, hipStream_t stream, Workspace& ws, SimArgs& a,
                      bool pwl_theta = false);
int launch_instances(const SimArgs& a, int n, int64_t N0, const Mlp* H, int prec,
                     const sl7_plan& plan, hipStream_t stream, Workspace& ws);
// The same launch sequence with its finalize scratch and statistics given
// directly (no workspace); enqueues kernels only.
int launch_sequence(const SimArgs& a, int n, int64_t N0, const Mlp* H, int prec,
                    const sl7_plan& plan, hipStream_t stream, int n_cu, void* chunks,
                    sl7_stats* stats);
int fill_nodes(int m, SimArgs& a, double* x_out);
void fill_inst(const sl7_problem& pr, const Mlp* H, const double* x, InstDev& I);
int run_instances(const sl7_problem* prs, int n, const Mlp* H, int prec, uint64_t seed,
                  void* YT_dev, const sl7_plan* plan, hipStream_t stream, Workspace& ws);
int fetch_stats(Workspace& ws, int n, sl7_stats* out, hipStream_t stream);

}  // namespace sl7
