// C ABI of the library (declared in include/sinkhorn.h): argument checks,
// workspace carving, launch planning and dispatch to the kernels.
#include "sk_internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

using namespace sk;

// Static device scratch of sinkhorn_solve_noalloc (one copy per device,
// held until the process ends).  In host code `scratch` names a host-side
// stand-in, never device memory: its device address is taken once per
// device with hipGetSymbolAddress and only that address is used.
constexpr size_t kNoAllocScratchBytes = (size_t)SK_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SK_EHIP;
  if (dev >= kMaxDevices) return SK_ENOTSUP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SK_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SK_OK;
}

inline hipStream_t S(sk_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

#define SK_HIP(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return SK_EHIP; \
  } while (0)

// ---------------------------------------------------------- Lambert W0
// Principal branch of the Lambert function for z >= 0 by Halley's method on
// f(w) = w e^w - z (Corless et al., "On the Lambert W function", 1996).
double lambert_w0(double z) {
  if (z == 0.0) return 0.0;
  double w;
  if (z < 1e-8) return z - z * z;            // series, error O(z^3)
  if (z <= M_E) w = log1p(z) * 0.75;         // start below the root
  else { const double L = log(z); w = L - log(L); }
  for (int it = 0; it < 100; ++it) {
    const double ew = exp(w);
    const double f = w * ew - z;
    const double wp1 = w + 1.0;
    const double step = f / (ew * wp1 - (w + 2.0) * f / (2.0 * wp1));
    w -= step;
    if (fabs(step) <= 1e-16 * (1.0 + fabs(w))) break;
  }
  return w;
}

// ---------------------------------------------------------- workspace
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    const size_t o = align_up(off, 256);
    off = o + align_up(sizeof(T) * count, 256);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

// One run of Algorithm 1 to schedule.
struct SolveSpec {
  const float *Prow, *Pcol, *a, *b, *srow, *scol;
  float *u, *v, *w, *z;
  sk_solve_info* info;
  int64_t n, m;
  int r;
  double eps;
};

// Per-process tuning: target feature bytes per workgroup of a solve, per
// solver class (indexed by the class's largest r).  Set by the autotuner.
std::map<int, int64_t>& tuning_table() {
  static std::map<int, int64_t> t;
  return t;
}

int class_rmax(int r) { return solver_class_rmax(r); }

// Lane layout variant per solver class (indexed like tuning_table); absent
// means variant 0.  Set by the autotuner.
std::map<int, int>& layout_table() {
  static std::map<int, int> t;
  return t;
}

constexpr int64_t kDefaultTarget = 256 * 1024;
constexpr int64_t kMaxRowsPerLane = 256;            // see run_solves
constexpr int64_t kSideBySideBytes = 256ll << 20;   // feature bytes per iteration

int planned_group(int64_t n, int64_t m, int r) {
  const int cls = class_rmax(r);
  int64_t target = kDefaultTarget;
  auto it = tuning_table().find(cls);
  if (it != tuning_table().end() && it->second > 0) target = it->second;
  const int64_t rows = n > m ? n : m;
  const int64_t bytes = rows * (int64_t)r * 4;
  int64_t g = (bytes + target - 1) / target;
  // precision floor (see run_solves): at most kMaxRowsPerLane rows per lane
  const int64_t per_wg = kMaxRowsPerLane * (int64_t)kBlock / std::max(solver_class_lanes(r), 1);
  g = std::max<int64_t>(g, (rows + per_wg - 1) / per_wg);
  if (g < 1) g = 1;
  if (g > kMaxGroup) g = kMaxGroup;
  // no more workgroups than row chunks of one wave-load each
  const int64_t min_rows = rows / 16 > 0 ? rows / 16 : 1;
  if (g > min_rows) g = min_rows;
  return (int)g;
}

// Lay out (and, when base != null and launch, run) a list of solves.  The
// same code computes the workspace size (base == null) and carves it, so
// the two can never disagree.
int run_solves(const std::vector<SolveSpec>& specs, const sk_solve_opts* o,
               void* base, size_t cap, size_t* need, hipStream_t s) {
  Carver cv(base);
  const int xr = o->range == SK_RANGE_EXTENDED ? 1 : 0;
  std::map<int, std::vector<int>> by_class;
  for (int i = 0; i < (int)specs.size(); ++i)
    by_class[class_rmax(specs[i].r)].push_back(i);
  std::vector<int> gplan(specs.size());
  int64_t max_sum_g = 0;
  int max_rmax = 4;
  for (auto& kv : by_class) {
    int64_t sg = 0;
    for (int i : kv.second) {
      gplan[i] = planned_group(specs[i].n, specs[i].m, specs[i].r);
      sg += gplan[i];
    }
    max_sum_g = std::max(max_sum_g, sg);
    max_rmax = std::max(max_rmax, kv.first);
  }
  // slots hold one partial r-vector per workgroup; pair layout [E | M] in
  // the extended range, so the stride is 2 * rmax for both domains
  const int64_t slot_count = std::min<int64_t>(kMaxGroup, max_sum_g);
  float* slots = cv.take<float>((size_t)slot_count * 2 * max_rmax);

  struct ClassBufs {
    LaunchCtl* ctl;
    unsigned* bars;
    SolveDesc* descs;
    int32_t* members;
    double* dpart;
  };
  std::map<int, ClassBufs> bufs;
  std::vector<float*> v2(specs.size()), w2(specs.size());
  for (auto& kv : by_class) {
    int64_t sg = 0;
    for (int i : kv.second) sg += gplan[i];
    ClassBufs cb;
    cb.ctl = cv.take<LaunchCtl>(1);
    cb.bars = cv.take<unsigned>(kv.second.size());
    cb.descs = cv.take<SolveDesc>(kv.second.size());
    cb.members = cv.take<int32_t>((size_t)sg);
    cb.dpart = cv.take<double>((size_t)sg * kDpartSlots);
    bufs[kv.first] = cb;
    for (int i : kv.second) {
      v2[i] = cv.take<float>(2 * (size_t)specs[i].m);
      w2[i] = cv.take<float>(2 * (size_t)specs[i].r);
    }
  }
  if (need) *need = cv.off;
  if (!base) return SK_OK;
  if (cv.off > cap) return SK_ENOMEM;

  for (auto& kv : by_class) {
    const int rmax = kv.first;
    int capdev = solver_capacity(rmax, xr);
    if (capdev <= 0) return SK_EHIP;
    capdev = std::min(capdev, kMaxGroup);
    std::vector<int> order = kv.second;
    // largest work first: seats are handed out in this order
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const int64_t wx = (specs[x].n + specs[x].m) * (int64_t)specs[x].r;
      const int64_t wy = (specs[y].n + specs[y].m) * (int64_t)specs[y].r;
      return wx > wy;
    });
    const ClassBufs& cb = bufs[rmax];
    // A solve starts once all of its g seats are taken, so workgroups that
    // take seats of a solve whose other seats are still held elsewhere wait.
    // The three solves of one divergence run one after the other on the
    // whole grid (their iteration counts differ, and a finished solve's
    // workgroups cannot join another).  A launch packing more solves gives
    // each a share of the grid proportional to its work per iteration, so
    // the gangs run side by side instead of queueing for the full grid.
    // Small solves are the exception: when one iteration streams at most
    // kSideBySideBytes (about the fixed cost of an iteration's barriers and
    // reductions at the full streaming rate), running them side by side
    // overlaps those fixed costs, which would otherwise be paid once per
    // solve.
    // Shares are rounded up: with T = total work / grid, a gang of
    // ceil(w / T) workgroups finishes within T, while rounding down could
    // stretch a large solve to nearly 2T and set the launch's length (the
    // workgroups of early finishers take the small solves' seats in turn).
    bool small = true;
    for (int i : order)
      small = small && 4 * (specs[i].n + specs[i].m) * (int64_t)specs[i].r <= kSideBySideBytes;
    // When the shares rounded up need more seats than the grid holds but the
    // shares rounded down (at least 1) do not, the seats are apportioned
    // instead (largest remainders first, Hamilton's method), so that every
    // gang starts at once: with rounded-up shares the last gang would have
    // members without a workgroup until a whole other solve finished (three
    // equal solves: 86 + 86 + 86 seats on 256 workgroups).
    std::vector<int> gshare(specs.size());
    if (order.size() > 3 || (order.size() > 1 && small)) {
      double total = 0.0;
      for (int i : order) total += (double)(specs[i].n + specs[i].m) * specs[i].r;
      int64_t sum_up = 0, sum_down = 0;
      std::vector<double> quota(specs.size());
      for (int i : order) {
        const double w = (double)(specs[i].n + specs[i].m) * specs[i].r;
        quota[i] = (double)capdev * w / total;
        const int64_t gi = (int64_t)ceil(quota[i]);
        gshare[i] = (int)std::max<int64_t>(1, std::min<int64_t>(gi, gplan[i]));
        sum_up += gshare[i];
        sum_down += std::max<int64_t>(1, std::min<int64_t>((int64_t)floor(quota[i]), gplan[i]));
      }
      if (sum_up > capdev && sum_down <= capdev) {
        int64_t left = capdev;
        for (int i : order) {
          gshare[i] = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)floor(quota[i]),
                                                                    gplan[i]));
          left -= gshare[i];
        }
        std::vector<int> byrem(order);
        std::stable_sort(byrem.begin(), byrem.end(), [&](int x, int y) {
          return quota[x] - floor(quota[x]) > quota[y] - floor(quota[y]);
        });
        for (int i : byrem) {
          if (left <= 0) break;
          if (gshare[i] < gplan[i] && (double)gshare[i] < quota[i]) {
            ++gshare[i];
            --left;
          }
        }
      }
    } else {
      for (int i : order) gshare[i] = gplan[i];
    }
    // Precision floor: each lane sums the transposed products of its rows
    // in float32, one after the other, so the rounding error of an r-vector
    // entry grows with the rows a lane adds (about sqrt(rows) units of
    // 2^-24).  That error changes from one iteration to the next and puts a
    // floor under the stop test's marginal error: a solve packed into a
    // small gang (two workgroups for 2e5 rows) stalled near 1e-6.  Every
    // gang is therefore large enough that no lane adds more than
    // kMaxRowsPerLane rows per half-step.
    const int lanes = solver_class_lanes(rmax);
    for (int i : order) {
      const int64_t rows = std::max(specs[i].n, specs[i].m);
      const int64_t per_wg = kMaxRowsPerLane * (int64_t)kBlock / std::max(lanes, 1);
      const int64_t gmin = (rows + per_wg - 1) / per_wg;   // <= gplan[i] by planning
      gshare[i] = (int)std::max<int64_t>(gshare[i], std::min<int64_t>(gmin, gplan[i]));
    }
    std::vector<SolveDesc> descs(order.size());
    int seat = 0;
    int64_t moff = 0;
    for (size_t k = 0; k < order.size(); ++k) {
      const int i = order[k];
      const SolveSpec& sp = specs[i];
      SolveDesc& D = descs[k];
      memset(&D, 0, sizeof(D));
      D.Prow = sp.Prow; D.Pcol = sp.Pcol; D.a = sp.a; D.b = sp.b;
      D.srow = sp.srow; D.scol = sp.scol;
      D.u = sp.u; D.v = sp.v; D.v2 = v2[i]; D.w = sp.w; D.w2 = w2[i]; D.z = sp.z;
      D.slots = slots;
      D.slot_stride = 2 * rmax;
      D.members = cb.members + moff;
      D.dpart = cb.dpart + kDpartSlots * moff;
      D.bar = cb.bars + k;
      D.info = sp.info;
      D.tol = o->tol;
      D.eps = sp.eps;
      D.n = sp.n; D.m = sp.m; D.r = sp.r;
      D.g = std::min(gshare[i], capdev);
      D.max_iter = o->max_iter;
      D.fixed_iter = o->fixed_iter;
      D.warm = o->warm_start;
      D.seat0 = seat;
      seat += D.g;
      moff += gplan[i];
    }
    const int grid = std::min(capdev, seat);
    SK_HIP(upload_descs(cb.descs, descs.data(), (int)descs.size(), s));
    SK_HIP(launch_init_ctl(cb.ctl, cb.bars, (int)descs.size(), s));
    SK_HIP(launch_solver(cb.descs, (int)descs.size(), rmax, xr, seat, grid,
                         cb.ctl, cb.bars, s));
  }
  return SK_OK;
}

// ---------------------------------------------------------- assembly
struct AsmDesc {
  const sk_solve_info* info;  // three consecutive records: xy, xx, yy
  double* state_out;          // double[4] in the state (may be null)
  double* out;                // double[4] of the caller (may be null)
  int32_t* meta;              // int32[4] in the state: [0] = numeric domain
  int32_t xr;
  int32_t pad;
};

// W_bar = W(mu,nu) - (W(mu,mu) + W(nu,nu)) / 2, Eq. (reg-sdiv), in float64.
__global__ void assemble_kernel(const AsmDesc* descs, AsmDesc one, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const AsmDesc D = descs ? descs[i] : one;
  const double wxy = D.info[0].w_hat, wxx = D.info[1].w_hat, wyy = D.info[2].w_hat;
  const double vals[4] = {wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy};
  for (int k = 0; k < 4; ++k) {
    if (D.state_out) D.state_out[k] = vals[k];
    if (D.out) D.out[k] = vals[k];
  }
  if (D.meta) {
    D.meta[0] = D.xr;
    D.meta[1] = 0;
    D.meta[2] = 0;
    D.meta[3] = 0;
  }
}

// The same for `count` problems whose three records are consecutive in
// `infos` (xy, xx, yy per problem): out[4i..4i+3] = {W_bar, W_xy, W_xx, W_yy}.
__global__ void assemble_strided_kernel(const sk_solve_info* infos, double* out, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double wxy = infos[3 * i].w_hat, wxx = infos[3 * i + 1].w_hat,
               wyy = infos[3 * i + 2].w_hat;
  out[4 * i] = wxy - 0.5 * (wxx + wyy);
  out[4 * i + 1] = wxy;
  out[4 * i + 2] = wxx;
  out[4 * i + 3] = wyy;
}

// Records the numeric domain in a state before its features are computed,
// so a backward pass always sees a defined flag.
__global__ void set_meta_kernel(int32_t* meta, int32_t xr) {
  if (threadIdx.x == 0) meta[0] = xr;
}

bool bad_ptr(const void* p) { return p == nullptr; }

int check_problem(const sk_problem* p) {
  if (!p) return SK_EINVAL;
  if (bad_ptr(p->X) || bad_ptr(p->Y) || bad_ptr(p->a) || bad_ptr(p->b) ||
      bad_ptr(p->U))
    return SK_EINVAL;
  if (p->n < 1 || p->m < 1 || p->d < 1 || p->r < 1) return SK_EINVAL;
  if (!(p->eps > 0.0) || !isfinite(p->eps)) return SK_EINVAL;
  if (!(p->q > 0.5) || !isfinite(p->q)) return SK_EINVAL;
  if (p->r > SK_MAX_R || p->r % 4 != 0) return SK_ENOTSUP;
  if (p->n > (int64_t)1 << 40 || p->m > (int64_t)1 << 40 || p->d > (1 << 20))
    return SK_EINVAL;
  return SK_OK;
}

// A divergence problem on arc-cosine features: q is not used; the solves
// see r + 1 columns, which the solver needs to be a multiple of 4.
int check_arccos_problem(const sk_problem* p) {
  if (!p) return SK_EINVAL;
  if (bad_ptr(p->X) || bad_ptr(p->Y) || bad_ptr(p->a) || bad_ptr(p->b) ||
      bad_ptr(p->U))
    return SK_EINVAL;
  if (p->n < 1 || p->m < 1 || p->d < 1 || p->r < 1) return SK_EINVAL;
  if (!(p->eps > 0.0) || !isfinite(p->eps)) return SK_EINVAL;
  if (p->r + 1 > SK_MAX_R || (p->r + 1) % 4 != 0) return SK_ENOTSUP;
  if (p->n > (int64_t)1 << 40 || p->m > (int64_t)1 << 40 || p->d > (1 << 20))
    return SK_EINVAL;
  return SK_OK;
}

int check_opts(const sk_solve_opts* o) {
  if (!o) return SK_EINVAL;
  if (!(o->tol >= 0.0)) return SK_EINVAL;
  if (o->fixed_iter < 0) return SK_EINVAL;
  if (o->fixed_iter == 0 && o->max_iter < 1) return SK_EINVAL;
  if (o->range != SK_RANGE_EXTENDED && o->range != SK_RANGE_LINEAR)
    return SK_EINVAL;
  return SK_OK;
}

void layout_of(int64_t n, int64_t m, int64_t r, sk_state_layout* L) {
  Carver cv(nullptr);
  auto at = [&](size_t bytes) {
    const size_t o = align_up(cv.off, 256);
    cv.off = o + align_up(bytes, 256);
    return o;
  };
  L->phix = at(4 * (size_t)n * r);
  L->phiy = at(4 * (size_t)m * r);
  L->sx = at(4 * (size_t)n);
  L->sy = at(4 * (size_t)m);
  // scalings and r-vectors are sized for the [E | M] pair layout
  const int64_t rows_u[3] = {n, n, m}, rows_v[3] = {m, n, m};
  for (int k = 0; k < 3; ++k) {
    L->u[k] = at(8 * (size_t)rows_u[k]);
    L->v[k] = at(8 * (size_t)rows_v[k]);
    L->w[k] = at(8 * (size_t)r);
    L->z[k] = at(8 * (size_t)r);
  }
  L->info = at(sizeof(sk_solve_info) * 3);
  L->out = at(sizeof(double) * 4);
  L->meta = at(sizeof(int32_t) * 4);
  L->total = align_up(cv.off, 256);
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}
template <typename T>
const T* at(const void* base, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

// The three solves of one divergence, reading/writing its state.
void divergence_specs(const sk_problem* p, void* state,
                      std::vector<SolveSpec>* out) {
  sk_state_layout L;
  layout_of(p->n, p->m, p->r, &L);
  const float* Px = at<float>(state, L.phix);
  const float* Py = at<float>(state, L.phiy);
  const float* sx = at<float>(state, L.sx);
  const float* sy = at<float>(state, L.sy);
  sk_solve_info* info = at<sk_solve_info>(state, L.info);
  const float* rows[3] = {Px, Px, Py};
  const float* cols[3] = {Py, Px, Py};
  const float* wa[3] = {p->a, p->a, p->b};
  const float* wb[3] = {p->b, p->a, p->b};
  const float* sr[3] = {sx, sx, sy};
  const float* sc[3] = {sy, sx, sy};
  const int64_t nr[3] = {p->n, p->n, p->m}, nc[3] = {p->m, p->n, p->m};
  for (int k = 0; k < 3; ++k) {
    SolveSpec sp;
    sp.Prow = rows[k]; sp.Pcol = cols[k]; sp.a = wa[k]; sp.b = wb[k];
    sp.srow = sr[k]; sp.scol = sc[k];
    sp.u = at<float>(state, L.u[k]);
    sp.v = at<float>(state, L.v[k]);
    sp.w = at<float>(state, L.w[k]);
    sp.z = at<float>(state, L.z[k]);
    sp.info = info + k;
    sp.n = nr[k]; sp.m = nc[k]; sp.r = (int)p->r; sp.eps = p->eps;
    out->push_back(sp);
  }
}

constexpr size_t kBackwardScratchDoubles = 4096;

int specs_from(const sk_solve_spec* in, int32_t count,
               std::vector<SolveSpec>* out) {
  if (!in || count < 1) return SK_EINVAL;
  for (int32_t i = 0; i < count; ++i) {
    const sk_solve_spec& p = in[i];
    if (!p.Prow || !p.Pcol || !p.a || !p.b || !p.u || !p.v || !p.w || !p.z ||
        !p.info)
      return SK_EINVAL;
    if (p.n < 1 || p.m < 1 || p.r < 1) return SK_EINVAL;
    if (!(p.eps > 0.0) || !isfinite(p.eps)) return SK_EINVAL;
    if (p.r > SK_MAX_R || p.r % 4 != 0) return SK_ENOTSUP;
    SolveSpec sp;
    sp.Prow = p.Prow; sp.Pcol = p.Pcol; sp.a = p.a; sp.b = p.b;
    sp.srow = p.srow; sp.scol = p.scol;
    sp.u = p.u; sp.v = p.v; sp.w = p.w; sp.z = p.z; sp.info = p.info;
    sp.n = p.n; sp.m = p.m; sp.r = (int)p.r; sp.eps = p.eps;
    out->push_back(sp);
  }
  return SK_OK;
}

}  // namespace

int sk::solver_layout_variant(int rmax) {
  auto it = layout_table().find(rmax);
  return it != layout_table().end() ? it->second : 0;
}

extern "C" {

const char* sinkhorn_strerror(int status) {
  switch (status) {
    case SK_OK: return "SK_OK";
    case SK_EINVAL: return "SK_EINVAL: invalid argument";
    case SK_ENOMEM: return "SK_ENOMEM: workspace or state buffer too small";
    case SK_ERANGE: return "SK_ERANGE: zero or non-finite value in a Sinkhorn division";
    case SK_ENOTCONV: return "SK_ENOTCONV: iteration cap reached before the tolerance";
    case SK_EHIP: return "SK_EHIP: HIP runtime error";
    case SK_ETIMEOUT: return "SK_ETIMEOUT: device-side wait exceeded its bound";
    case SK_ENOTSUP: return "SK_ENOTSUP: unsupported shape";
    default: return "unknown status";
  }
}

const char* sinkhorn_version(void) { return "paper_2006_07057_amd 0.1 (gfx950)"; }

int sinkhorn_gaussian_q(double R, double eps, int64_t d, double* q_host) {
  if (!q_host || !(R > 0.0) || !(eps > 0.0) || d < 1 || !isfinite(R) ||
      !isfinite(eps))
    return SK_EINVAL;
  const double z = R * R / (eps * (double)d);
  const double w = lambert_w0(z);
  // q = z / (2 W0(z)); for tiny z, W0(z) ~ z and q -> 1/2
  *q_host = (z < 1e-8) ? 0.5 / (1.0 - z) : z / (2.0 * w);
  return SK_OK;
}

int sinkhorn_features(const float* X, int64_t n, int64_t d, const float* U,
                      int64_t r, double eps, double q, int32_t range,
                      float* Phi, float* logscale, sk_stream_t stream) {
  if (!X || !U || !Phi || !logscale || n < 1 || d < 1 || r < 1) return SK_EINVAL;
  if (!(eps > 0.0) || !(q > 0.5) || !isfinite(eps) || !isfinite(q))
    return SK_EINVAL;
  if (range != SK_RANGE_EXTENDED && range != SK_RANGE_LINEAR) return SK_EINVAL;
  if (r > SK_MAX_R) return SK_ENOTSUP;
  if (d > (1 << 20) || n > (int64_t)1 << 40) return SK_EINVAL;
  SK_HIP(launch_features(X, n, (int)d, U, (int)r, eps, q,
                         range == SK_RANGE_EXTENDED ? 1 : 0, Phi, logscale,
                         S(stream)));
  return SK_OK;
}

int sinkhorn_features_arccos(const float* X, int64_t n, int64_t d, const float* U,
                             int64_t r, int32_t s_exp, double sigma, double kappa,
                             float* Phi, float* logscale, sk_stream_t stream) {
  if (!X || !U || !Phi || !logscale || n < 1 || d < 1 || r < 1) return SK_EINVAL;
  if (s_exp < 0 || s_exp > 8) return SK_EINVAL;
  if (!(sigma > 1.0) || !(kappa > 0.0) || !isfinite(sigma) || !isfinite(kappa))
    return SK_EINVAL;
  if (r + 1 > SK_MAX_R) return SK_ENOTSUP;
  if (d > (1 << 20) || n > (int64_t)1 << 40) return SK_EINVAL;
  SK_HIP(launch_features_arccos(X, n, (int)d, U, (int)r, s_exp, sigma, kappa, Phi,
                                logscale, S(stream)));
  return SK_OK;
}

size_t sinkhorn_solve_workspace_size(int64_t n, int64_t m, int64_t r) {
  if (n < 1 || m < 1 || r < 1 || r > SK_MAX_R) return 0;
  std::vector<SolveSpec> specs(1);
  memset(&specs[0], 0, sizeof(SolveSpec));
  specs[0].n = n; specs[0].m = m; specs[0].r = (int)r;
  size_t need = 0;
  sk_solve_opts o{};
  o.max_iter = 1;
  run_solves(specs, &o, nullptr, 0, &need, nullptr);
  return need;
}

int sinkhorn_solve(const float* Phix, int64_t n, const float* Phiy, int64_t m,
                   int64_t r, const float* a, const float* b,
                   const sk_solve_opts* opts, float* u, float* v, float* w,
                   float* z, sk_solve_info* info, void* ws, size_t ws_bytes,
                   sk_stream_t stream) {
  if (!Phix || !Phiy || !a || !b || !u || !v || !w || !z || !info || !ws)
    return SK_EINVAL;
  if (n < 1 || m < 1 || r < 1) return SK_EINVAL;
  if (r > SK_MAX_R || r % 4 != 0) return SK_ENOTSUP;
  int rc = check_opts(opts);
  if (rc) return rc;
  SolveSpec sp;
  sp.Prow = Phix; sp.Pcol = Phiy; sp.a = a; sp.b = b;
  sp.srow = nullptr; sp.scol = nullptr;
  sp.u = u; sp.v = v; sp.w = w; sp.z = z; sp.info = info;
  sp.n = n; sp.m = m; sp.r = (int)r; sp.eps = 1.0;
  std::vector<SolveSpec> specs{sp};
  size_t need = 0;
  return run_solves(specs, opts, ws, ws_bytes, &need, S(stream));
}

int sinkhorn_solve_noalloc(const float* Phix, int64_t n, const float* Phiy, int64_t m,
                           int64_t r, const float* a, const float* b,
                           const sk_solve_opts* opts, float* u, float* v, float* w,
                           float* z, sk_solve_info* info, sk_stream_t stream) {
  if (!Phix || !Phiy || !a || !b || !u || !v || !w || !z || !info) return SK_EINVAL;
  if (n < 1 || m < 1 || r < 1) return SK_EINVAL;
  if (r > SK_MAX_R || r % 4 != 0) return SK_ENOTSUP;
  int rc = check_opts(opts);
  if (rc) return rc;
  SolveSpec sp;
  sp.Prow = Phix; sp.Pcol = Phiy; sp.a = a; sp.b = b;
  sp.srow = nullptr; sp.scol = nullptr;
  sp.u = u; sp.v = v; sp.w = w; sp.z = z; sp.info = info;
  sp.n = n; sp.m = m; sp.r = (int)r; sp.eps = 1.0;
  std::vector<SolveSpec> specs{sp};
  size_t need = 0;
  run_solves(specs, opts, nullptr, 0, &need, nullptr);
  if (need > kNoAllocScratchBytes) return SK_ENOMEM;
  void* ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc) return rc;
  // every piece of the workspace that must start at zero (launch control
  // block, barrier counters) is cleared by the launch sequence itself
  return run_solves(specs, opts, ws, kNoAllocScratchBytes, &need, S(stream));
}

size_t sinkhorn_solve_batched_workspace_size(const sk_solve_spec* specs,
                                             int32_t count) {
  std::vector<SolveSpec> v;
  if (specs_from(specs, count, &v) != SK_OK) return 0;
  size_t need = 0;
  sk_solve_opts o{};
  o.max_iter = 1;
  run_solves(v, &o, nullptr, 0, &need, nullptr);
  return need;
}

int sinkhorn_solve_batched(const sk_solve_spec* specs, int32_t count,
                           const sk_solve_opts* opts, void* ws,
                           size_t ws_bytes, sk_stream_t stream) {
  std::vector<SolveSpec> v;
  int rc = specs_from(specs, count, &v);
  if (rc) return rc;
  rc = check_opts(opts);
  if (rc) return rc;
  if (!ws) return SK_EINVAL;
  size_t need = 0;
  return run_solves(v, opts, ws, ws_bytes, &need, S(stream));
}

size_t sinkhorn_solve_accelerated_workspace_size(const sk_solve_spec* spec) {
  std::vector<SolveSpec> sp;
  if (specs_from(spec, 1, &sp) != SK_OK) return 0;
  const int g = accel_planned_group(sp[0].n, sp[0].m, sp[0].r);
  return accel_workspace_bytes(sp[0].n, sp[0].m, sp[0].r, g);
}

int sinkhorn_solve_accelerated(const sk_solve_spec* spec, const sk_solve_opts* opts,
                               double L0, int32_t* trials, void* ws, size_t ws_bytes,
                               sk_stream_t stream) {
  std::vector<SolveSpec> sp;
  int rc = specs_from(spec, 1, &sp);
  if (rc != SK_OK) return rc;
  if ((rc = check_opts(opts)) != SK_OK) return rc;
  if (!(L0 > 0.0) || !isfinite(L0)) return SK_EINVAL;
  if (opts->range != SK_RANGE_LINEAR || opts->warm_start) return SK_ENOTSUP;
  if (!ws) return SK_EINVAL;
  const SolveSpec& p = sp[0];
  const int g = accel_planned_group(p.n, p.m, p.r);
  if (ws_bytes < accel_workspace_bytes(p.n, p.m, p.r, g)) return SK_ENOMEM;
  SK_HIP(launch_accelerated(p.Prow, p.Pcol, p.a, p.b, p.srow, p.scol, p.u, p.v, p.w,
                            p.z, p.info, trials, p.n, p.m, p.r, p.eps, opts->tol,
                            opts->max_iter, opts->fixed_iter, L0, ws, g, S(stream)));
  return SK_OK;
}

size_t sinkhorn_divergence_accelerated_workspace_size(const sk_problem* p) {
  if (check_problem(p) != SK_OK) return 0;
  size_t need = 0;
  const int64_t nr[3] = {p->n, p->n, p->m}, nc[3] = {p->m, p->n, p->m};
  for (int k = 0; k < 3; ++k) {
    const int g = accel_planned_group(nr[k], nc[k], (int)p->r);
    need = std::max(need, accel_workspace_bytes(nr[k], nc[k], (int)p->r, g));
  }
  return need;
}

int sinkhorn_divergence_accelerated(const sk_problem* p, const sk_solve_opts* opts,
                                    double L0, double* out, void* state,
                                    size_t state_bytes, void* ws, size_t ws_bytes,
                                    sk_stream_t stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  rc = check_opts(opts);
  if (rc) return rc;
  if (!(L0 > 0.0) || !isfinite(L0)) return SK_EINVAL;
  if (opts->range != SK_RANGE_LINEAR || opts->warm_start) return SK_ENOTSUP;
  if (!state || !ws) return SK_EINVAL;
  sk_state_layout L;
  layout_of(p->n, p->m, p->r, &L);
  if (state_bytes < L.total) return SK_ENOMEM;
  if (ws_bytes < sinkhorn_divergence_accelerated_workspace_size(p)) return SK_ENOMEM;
  hipStream_t s = S(stream);
  int32_t* meta = at<int32_t>(state, L.meta);
  hipLaunchKernelGGL(set_meta_kernel, dim3(1), dim3(64), 0, s, meta, 0);
  SK_HIP(hipGetLastError());
  SK_HIP(launch_features_pair(p->X, p->n, p->Y, p->m, (int)p->d, p->U, (int)p->r, p->eps,
                              p->q, 0, at<float>(state, L.phix), at<float>(state, L.sx),
                              at<float>(state, L.phiy), at<float>(state, L.sy), s));
  std::vector<SolveSpec> specs;
  divergence_specs(p, state, &specs);
  // the three solves run one after the other, reusing the workspace
  for (int k = 0; k < 3; ++k) {
    const SolveSpec& q = specs[k];
    const int g = accel_planned_group(q.n, q.m, q.r);
    SK_HIP(launch_accelerated(q.Prow, q.Pcol, q.a, q.b, q.srow, q.scol, q.u, q.v, q.w,
                              q.z, q.info, meta + 1 + k, q.n, q.m, q.r, q.eps, opts->tol,
                              opts->max_iter, opts->fixed_iter, L0, ws, g, s));
  }
  AsmDesc one{at<sk_solve_info>(state, L.info), at<double>(state, L.out), out, nullptr,
              0, 0};
  hipLaunchKernelGGL(assemble_kernel, dim3(1), dim3(64), 0, s, nullptr, one, 1);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int sinkhorn_divergence_assemble(const sk_solve_info* infos, int32_t count, double* out,
                                 sk_stream_t stream) {
  if (!infos || !out || count < 1) return SK_EINVAL;
  hipLaunchKernelGGL(assemble_strided_kernel, dim3((count + 63) / 64), dim3(64), 0,
                     S(stream), infos, out, count);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int sinkhorn_gaussian_anchors(const double* Z_host, int64_t r, int64_t d, double eps,
                              double sigma2, double R, float* U_host, double* q_host) {
  if (!Z_host || !U_host || !q_host || r < 1 || d < 1) return SK_EINVAL;
  if (!(eps > 0.0) || !isfinite(eps)) return SK_EINVAL;
  double q;
  if (sigma2 > 0.0) {
    if (!isfinite(sigma2)) return SK_EINVAL;
    q = 4.0 * sigma2 / eps;              // sigma^2 = q eps / 4 (Lemma 1)
  } else {
    const int rc = sinkhorn_gaussian_q(R, eps, d, &q);
    if (rc != SK_OK) return rc;
    sigma2 = q * eps / 4.0;
  }
  const double sigma = sqrt(sigma2);
  for (int64_t i = 0; i < r * d; ++i) U_host[i] = (float)(sigma * Z_host[i]);
  *q_host = q;
  return SK_OK;
}

size_t sinkhorn_divergence_arccos_workspace_size(const sk_problem* p) {
  if (check_arccos_problem(p) != SK_OK) return 0;
  sk_problem q = *p;
  q.r = p->r + 1;
  std::vector<SolveSpec> specs;
  divergence_specs(&q, nullptr, &specs);
  size_t need = 0;
  sk_solve_opts o{};
  o.max_iter = 1;
  o.range = SK_RANGE_LINEAR;
  run_solves(specs, &o, nullptr, 0, &need, nullptr);
  return need;
}

int sinkhorn_divergence_arccos(const sk_problem* p, int32_t s_exp, double sigma,
                               double kappa, const sk_solve_opts* opts, double* out,
                               void* state, size_t state_bytes, void* ws, size_t ws_bytes,
                               sk_stream_t stream) {
  int rc = check_arccos_problem(p);
  if (rc) return rc;
  rc = check_opts(opts);
  if (rc) return rc;
  if (opts->range != SK_RANGE_LINEAR) return SK_ENOTSUP;
  if (s_exp < 0 || s_exp > 8) return SK_EINVAL;
  if (!(sigma > 1.0) || !(kappa > 0.0) || !isfinite(sigma) || !isfinite(kappa))
    return SK_EINVAL;
  if (!state || !ws) return SK_EINVAL;
  sk_problem q = *p;          // the solves see r + 1 feature columns
  q.r = p->r + 1;
  sk_state_layout L;
  layout_of(q.n, q.m, q.r, &L);
  if (state_bytes < L.total) return SK_ENOMEM;
  if (ws_bytes < sinkhorn_divergence_arccos_workspace_size(p)) return SK_ENOMEM;
  hipStream_t s = S(stream);
  int32_t* meta = at<int32_t>(state, L.meta);
  hipLaunchKernelGGL(set_meta_kernel, dim3(1), dim3(64), 0, s, meta, 0);
  SK_HIP(hipGetLastError());
  SK_HIP(launch_features_arccos(p->X, p->n, (int)p->d, p->U, (int)p->r, s_exp, sigma, kappa,
                                at<float>(state, L.phix), at<float>(state, L.sx), s));
  SK_HIP(launch_features_arccos(p->Y, p->m, (int)p->d, p->U, (int)p->r, s_exp, sigma, kappa,
                                at<float>(state, L.phiy), at<float>(state, L.sy), s));
  std::vector<SolveSpec> specs;
  divergence_specs(&q, state, &specs);
  size_t need = 0;
  rc = run_solves(specs, opts, ws, ws_bytes, &need, s);
  if (rc) return rc;
  AsmDesc one{at<sk_solve_info>(state, L.info), at<double>(state, L.out), out, meta, 0, 0};
  hipLaunchKernelGGL(assemble_kernel, dim3(1), dim3(64), 0, s, nullptr, one, 1);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int sinkhorn_tune_set(int64_t r, int64_t target_bytes) {
  if (r < 1 || r > SK_MAX_R || target_bytes < 0) return SK_EINVAL;
  const int cls = class_rmax((int)r);
  if (cls <= 0) return SK_EINVAL;
  if (target_bytes == 0) tuning_table().erase(cls);
  else tuning_table()[cls] = target_bytes;
  return SK_OK;
}

int64_t sinkhorn_tune_get(int64_t r) {
  if (r < 1 || r > SK_MAX_R) return -1;
  const int cls = class_rmax((int)r);
  if (cls <= 0) return -1;
  auto it = tuning_table().find(cls);
  return it != tuning_table().end() ? it->second : kDefaultTarget;
}

int32_t sinkhorn_solver_layouts(int64_t r, int32_t* out, int32_t max) {
  if (r < 1 || r > SK_MAX_R || max < 0) return SK_EINVAL;
  return solver_layouts((int)r, out, max);
}

int sinkhorn_tune_set_layout(int64_t r, int32_t variant) {
  if (r < 1 || r > SK_MAX_R) return SK_EINVAL;
  const int cls = class_rmax((int)r);
  if (cls <= 0 || variant < 0 || variant >= solver_layouts((int)r, nullptr, 0))
    return SK_EINVAL;
  if (variant == 0) layout_table().erase(cls);
  else layout_table()[cls] = variant;
  return SK_OK;
}

int32_t sinkhorn_tune_get_layout(int64_t r) {
  if (r < 1 || r > SK_MAX_R) return -1;
  const int cls = class_rmax((int)r);
  if (cls <= 0) return -1;
  return solver_layout_variant(cls);
}

int sinkhorn_state_layout(int64_t n, int64_t m, int64_t r,
                          sk_state_layout* layout) {
  if (!layout || n < 1 || m < 1 || r < 1) return SK_EINVAL;
  layout_of(n, m, r, layout);
  return SK_OK;
}

size_t sinkhorn_divergence_workspace_size(const sk_problem* p) {
  if (check_problem(p) != SK_OK) return 0;
  std::vector<SolveSpec> specs;
  divergence_specs(p, nullptr, &specs);
  size_t need = 0;
  sk_solve_opts o{};
  o.max_iter = 1;
  run_solves(specs, &o, nullptr, 0, &need, nullptr);
  return std::max(need, kBackwardScratchDoubles * sizeof(double));
}

int sinkhorn_divergence(const sk_problem* p, const sk_solve_opts* opts,
                        double* out, void* state, size_t state_bytes, void* ws,
                        size_t ws_bytes, sk_stream_t stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  rc = check_opts(opts);
  if (rc) return rc;
  if (!state || !ws) return SK_EINVAL;
  sk_state_layout L;
  layout_of(p->n, p->m, p->r, &L);
  if (state_bytes < L.total) return SK_ENOMEM;
  if (ws_bytes < sinkhorn_divergence_workspace_size(p)) return SK_ENOMEM;
  hipStream_t s = S(stream);
  const int xr = opts->range == SK_RANGE_EXTENDED ? 1 : 0;
  hipLaunchKernelGGL(set_meta_kernel, dim3(1), dim3(64), 0, s,
                     at<int32_t>(state, L.meta), xr);
  SK_HIP(hipGetLastError());
  SK_HIP(launch_features_pair(p->X, p->n, p->Y, p->m, (int)p->d, p->U, (int)p->r, p->eps,
                              p->q, xr, at<float>(state, L.phix), at<float>(state, L.sx),
                              at<float>(state, L.phiy), at<float>(state, L.sy), s));
  std::vector<SolveSpec> specs;
  divergence_specs(p, state, &specs);
  size_t need = 0;
  rc = run_solves(specs, opts, ws, ws_bytes, &need, s);
  if (rc) return rc;
  AsmDesc one{at<sk_solve_info>(state, L.info), at<double>(state, L.out), out,
              at<int32_t>(state, L.meta), xr, 0};
  hipLaunchKernelGGL(assemble_kernel, dim3(1), dim3(64), 0, s, nullptr, one, 1);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

size_t sinkhorn_batched_workspace_size(const sk_problem* problems,
                                       int32_t count) {
  if (!problems || count < 1) return 0;
  std::vector<SolveSpec> specs;
  for (int i = 0; i < count; ++i) {
    if (check_problem(&problems[i]) != SK_OK) return 0;
    divergence_specs(&problems[i], nullptr, &specs);
  }
  size_t need = 0;
  sk_solve_opts o{};
  o.max_iter = 1;
  run_solves(specs, &o, nullptr, 0, &need, nullptr);
  // feature descriptors + assembly descriptors after the solver's part
  need = align_up(need, 256) + align_up(sizeof(FeatDesc) * 2 * (size_t)count, 256) +
         align_up(sizeof(AsmDesc) * (size_t)count, 256);
  return std::max(need, kBackwardScratchDoubles * sizeof(double));
}

int sinkhorn_divergence_batched(const sk_problem* problems, int32_t count,
                                const sk_solve_opts* opts, double* out,
                                void* const* states, void* ws, size_t ws_bytes,
                                sk_stream_t stream) {
  if (!problems || count < 1 || !states || !ws) return SK_EINVAL;
  int rc = check_opts(opts);
  if (rc) return rc;
  for (int i = 0; i < count; ++i) {
    rc = check_problem(&problems[i]);
    if (rc) return rc;
    if (!states[i]) return SK_EINVAL;
  }
  if (ws_bytes < sinkhorn_batched_workspace_size(problems, count)) return SK_ENOMEM;
  hipStream_t s = S(stream);
  std::vector<SolveSpec> specs;
  for (int i = 0; i < count; ++i) divergence_specs(&problems[i], states[i], &specs);
  size_t need = 0;
  run_solves(specs, opts, nullptr, 0, &need, nullptr);
  char* tail = static_cast<char*>(ws) + align_up(need, 256);
  FeatDesc* fdev = reinterpret_cast<FeatDesc*>(tail);
  AsmDesc* adev = reinterpret_cast<AsmDesc*>(
      tail + align_up(sizeof(FeatDesc) * 2 * (size_t)count, 256));

  // features: group the 2*count clouds by feature class, one launch each
  const int xr = opts->range == SK_RANGE_EXTENDED ? 1 : 0;
  std::map<int, std::vector<FeatDesc>> fgroups;
  for (int i = 0; i < count; ++i) {
    const sk_problem& p = problems[i];
    sk_state_layout L;
    layout_of(p.n, p.m, p.r, &L);
    FeatDesc fx{p.X, p.U, at<float>(states[i], L.phix), at<float>(states[i], L.sx),
                p.n, (int32_t)p.d, (int32_t)p.r, p.eps, p.q, xr, 0, 0};
    FeatDesc fy{p.Y, p.U, at<float>(states[i], L.phiy), at<float>(states[i], L.sy),
                p.m, (int32_t)p.d, (int32_t)p.r, p.eps, p.q, xr, 0, 0};
    fgroups[class_rmax((int)p.r)].push_back(fx);
    fgroups[class_rmax((int)p.r)].push_back(fy);
  }
  FeatDesc* fcur = fdev;
  for (auto& kv : fgroups) {
    SK_HIP(launch_features_batched(kv.second.data(), (int)kv.second.size(), fcur, s));
    fcur += kv.second.size();
  }
  rc = run_solves(specs, opts, ws, ws_bytes, &need, s);
  if (rc) return rc;
  std::vector<AsmDesc> ad(count);
  for (int i = 0; i < count; ++i) {
    const sk_problem& p = problems[i];
    sk_state_layout L;
    layout_of(p.n, p.m, p.r, &L);
    ad[i] = AsmDesc{at<sk_solve_info>(states[i], L.info),
                    at<double>(states[i], L.out), out ? out + 4 * i : nullptr,
                    at<int32_t>(states[i], L.meta), xr, 0};
  }
  SK_HIP(upload_bytes(adev, ad.data(), sizeof(AsmDesc) * ad.size(), s));
  hipLaunchKernelGGL(assemble_kernel, dim3((count + 63) / 64), dim3(64), 0, s,
                     adev, ad[0], count);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int sinkhorn_features_backward(const float* X, int64_t n, int64_t d,
                               const float* U, int64_t r, const float* Phi,
                               const float* p, const float* g, float coef,
                               int32_t accumulate, int32_t range, float* dX,
                               sk_stream_t stream) {
  if (!X || !U || !Phi || !p || !g || !dX || n < 1 || d < 1 || r < 1)
    return SK_EINVAL;
  if (range != SK_RANGE_EXTENDED && range != SK_RANGE_LINEAR) return SK_EINVAL;
  if (r > SK_MAX_R || r % 4 != 0) return SK_ENOTSUP;
  SK_HIP(launch_features_backward(X, n, (int)d, U, (int)r, Phi, p, g, coef,
                                  nullptr, nullptr, 0.f, nullptr, nullptr, 0.f,
                                  nullptr, accumulate, nullptr,
                                  range == SK_RANGE_EXTENDED ? 1 : 0, dX,
                                  S(stream)));
  return SK_OK;
}

int sinkhorn_divergence_backward(const sk_problem* p, const void* state,
                                 const float* grad_out, float* dX, float* da,
                                 float* dY, float* db, void* ws,
                                 size_t ws_bytes, sk_stream_t stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (!state) return SK_EINVAL;
  if ((da || db) && (!ws || ws_bytes < kBackwardScratchDoubles * sizeof(double)))
    return SK_ENOMEM;
  sk_state_layout L;
  layout_of(p->n, p->m, p->r, &L);
  hipStream_t s = S(stream);
  const float* u[3];
  const float* v[3];
  const float* w[3];
  const float* z[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = at<float>(state, L.u[k]);
    v[k] = at<float>(state, L.v[k]);
    w[k] = at<float>(state, L.w[k]);
    z[k] = at<float>(state, L.z[k]);
  }
  const int r = (int)p->r, d = (int)p->d;
  // the numeric domain recorded by the forward call, read on the device
  const int32_t* xf = at<int32_t>(state, L.meta);
  if (dX)
    SK_HIP(launch_features_backward(p->X, p->n, d, p->U, r,
                                    at<float>(state, L.phix), u[0], w[0], 1.0f,
                                    u[1], w[1], -0.5f, v[1], z[1], -0.5f,
                                    grad_out, 0, xf, 0, dX, s));
  if (dY)
    SK_HIP(launch_features_backward(p->Y, p->m, d, p->U, r,
                                    at<float>(state, L.phiy), v[0], z[0], 1.0f,
                                    u[2], w[2], -0.5f, v[2], z[2], -0.5f,
                                    grad_out, 0, xf, 0, dY, s));
  double* scratch = static_cast<double*>(ws);
  const int half = (int)kBackwardScratchDoubles / 2;
  if (da)
    SK_HIP(launch_weight_grad(u[0], u[1], v[1], p->n, p->eps, grad_out, xf,
                              scratch, half, da, s));
  if (db)
    SK_HIP(launch_weight_grad(v[0], u[2], v[2], p->m, p->eps, grad_out, xf,
                              scratch + half, half, db, s));
  return SK_OK;
}

size_t sinkhorn_divergence_backward_anchors_workspace_size(const sk_problem* p) {
  if (check_problem(p) != SK_OK) return 0;
  return anchor_grad_scratch_floats((int)p->r, (int)p->d, p->n, p->m) * sizeof(float);
}

int sinkhorn_divergence_backward_anchors(const sk_problem* p, const void* state,
                                         const float* grad_out, float* dU, void* ws,
                                         size_t ws_bytes, sk_stream_t stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (!state || !dU || !ws) return SK_EINVAL;
  if (ws_bytes < anchor_grad_scratch_floats((int)p->r, (int)p->d, p->n, p->m) * sizeof(float))
    return SK_ENOMEM;
  sk_state_layout L;
  layout_of(p->n, p->m, p->r, &L);
  const float* u[3];
  const float* v[3];
  const float* w[3];
  const float* z[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = at<float>(state, L.u[k]);
    v[k] = at<float>(state, L.v[k]);
    w[k] = at<float>(state, L.w[k]);
    z[k] = at<float>(state, L.z[k]);
  }
  SK_HIP(launch_anchor_grad(p->X, p->n, p->Y, p->m, (int)p->d, p->U, (int)p->r, p->q,
                            at<float>(state, L.phix), at<float>(state, L.phiy), u, v, w,
                            z, grad_out, at<int32_t>(state, L.meta),
                            static_cast<float*>(ws), dU, S(stream)));
  return SK_OK;
}

}  // extern "C"
