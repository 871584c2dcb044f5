// Batch engine: restarted FGMRES over a changing set of independent KKT
// systems (slots), advanced together one cycle at a time.
#pragma once

#include <chrono>
#include <map>
#include <memory>

#include "coarse.hpp"
#include "ras.hpp"

namespace stkkt {

struct PinnedBlock {
  void *p = nullptr;
  explicit PinnedBlock(size_t bytes);
  ~PinnedBlock();
  PinnedBlock(const PinnedBlock &) = delete;
  PinnedBlock &operator=(const PinnedBlock &) = delete;
  template <class T> T *as() const { return static_cast<T *>(p); }
};

class BatchEngine {
 public:
  // capacity: elements of the concatenated vectors; slots: most members at once
  BatchEngine(const Allocator *al, const solve_params_t &sp, long long capacity, int slots, hipStream_t s);

  // Reserve a slot for one system (two-level when C != NULL).  Returns the
  // slot, or -1 when the slots or the vector capacity are exhausted.  The
  // caller then fills b_of(slot) and x_of(slot) (x0) on the engine's stream.
  int admit(const kkt_op *op, const ras *R, const coarse *C);
  double *b_of(int slot) const { return B_.as<double>() + slots_[slot].voff; }
  double *x_of(int slot) const { return X_.as<double>() + slots_[slot].voff; }
  long long size_of(int slot) const { return slots_[slot].n; }

  // Initial residuals of newly admitted members, then one FGMRES cycle of
  // every running member; members that converge, reach maxit or break down
  // are appended to `finished` (their x_of() holds the result until release).
  void cycle(std::vector<int> &finished);
  const kkt_stats_t &stats(int slot) const { return slots_[slot].st; }
  void release(int slot);

  int active() const { return nused_; }
  int slots() const { return (int)slots_.size(); }
  long long capacity() const { return cap_; }
  long long free_elems() const;
  // bytes of device memory a member with n unknowns takes besides its share of the vectors
  static size_t member_bytes(const kkt_op *op, const ras *R, const coarse *C);

 private:
  struct Slot {
    bool used = false;
    const kkt_op *op = nullptr;
    const ras *R = nullptr;
    const coarse *C = nullptr;
    long long voff = 0, n = 0;
    DevBuf local, y2;
    int state = 0;   // 0 new, 1 running, 2 finished
    bool breakdown = false;
    double bnorm = 0, target = 0, beta = 0;
    kkt_stats_t st{};
    std::vector<double> Hm, g, cs, sn;
    int kdone = 0;
    std::chrono::steady_clock::time_point t0;
  };
  void rebuild();
  void drop_graphs();
  void cgs2(int j, const int *act);
  void arnoldi_step(int j);   // the device-only step of the graph form (flags in act_a_)
  void cycle_graph(const int *run, int S);
  void upload(int *host, DevBuf &dev);
  void bdot(const double *V, long long ldv, int k, const double *w, const int *act, double *out);
  void fetch();
  void precondition(int j, const int *act_dev);

  const Allocator *al_;
  solve_params_t sp_;
  hipStream_t s_;
  long long cap_;
  int m_, hs_;
  std::vector<Slot> slots_;
  int nused_ = 0;
  bool dirty_ = true;
  std::map<long long, long long> free_;   // start -> length
  DevBuf V_, Z_, B_, X_, R_, W_, T_, partial_, hdev_, ydev_, chunks_, cfirst_, kcnt_;
  DevBuf act_a_, act_b_, act_c_;
  std::unique_ptr<PinnedBlock> hh_, hy_, hflags_;
  int nch_ = 0;
  MvBatch mv_;
  RasBatch rb_;
  // graph form: per slot cs[m], sn[m], g[m+1], H[(m+1) m] (gst_), iters,
  // kdone, breakdown, spare (gin_), target (gtg_); captured step graphs of
  // the current composition (kGraphSteps steps each), captured on cs_
  DevBuf gst_, gin_, gtg_;
  std::unique_ptr<PinnedBlock> hg_;
  hipStream_t cs_ = nullptr;
  std::vector<hipGraphExec_t> graphs_;
  long long gstride_ = 0;
 public:
  ~BatchEngine();
  BatchEngine(const BatchEngine &) = delete;
  BatchEngine &operator=(const BatchEngine &) = delete;
};

}  // namespace stkkt
