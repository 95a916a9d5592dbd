// Allocation-free field synthesis (scw_synthesize_noalloc): the kernels of
// scw_synthesize with every table and workspace in one static device array.
//
// The plan tables that scw_synthesize builds on the host and uploads (the
// interior plane tasks with their z offsets, the exterior plane list, the
// transform twiddles) are built here by two kernels on the caller's stream,
// so the call neither allocates nor copies from the host, and can be
// captured in a HIP graph. The plane classification repeats the host rule of
// classify_plane operation by operation, in correctly rounded double
// arithmetic without contraction, so both put every plane in the same layer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "scw_internal.h"

// One copy per GPU (each device that loads the library holds its own), kept
// until the process ends. Host code never passes this name to a kernel or a
// copy: it uses the per-device address taken by noalloc_attach.
static __device__ __align__(256) unsigned char scratch[SCW_NOALLOC_SCRATCH_BYTES];

namespace scw {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_attach_lock;
void* g_scratch_ptr[kMaxDevices] = {};

struct DevPlane {
  int kind, layer;
  double dz_top, dz_bot;
};

// classify_plane on the device: z = z_begin + (j + 1/2) (z_end - z_begin) / fz.
__device__ DevPlane dev_classify(double z_begin, double z_end, int fz, int L, double d, int j) {
  const double zL = __dmul_rn((double)L, d);
  const double dz = __ddiv_rn(__dadd_rn(z_end, -z_begin), (double)fz);
  const double z = __dadd_rn(z_begin, __dmul_rn((double)j + 0.5, dz));
  if (z < 0.0) return {0, -1, z, 0.0};
  if (z >= zL) return {2, L, __dadd_rn(z, -zL), 0.0};
  const int l = min((int)floor(__ddiv_rn(z, d)), L - 1);
  return {1, l, __dadd_rn(z, -__dmul_rn((double)l, d)),
          __dadd_rn(z, -__dmul_rn((double)(l + 1), d))};
}

__device__ int load_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One block of 1024 threads: per-layer first plane and plane count, then the
// task and exterior tables in plane order (a chunked exclusive scan of the
// per-thread counts gives every entry its index).
__global__ void __launch_bounds__(1024)
noalloc_planes_kernel(double z_begin, double z_end, int fz, int L, double d, int zt,
                      int ntasks, int n_ext_max, int* __restrict__ first, int* __restrict__ count, Task* __restrict__ tasks,
                      double* __restrict__ task_dz, float* __restrict__ task_dz32,
                      ExtPlane* __restrict__ ext) {
  __shared__ int s_task[1024], s_ext[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = tid; l < L; l += nt) {
    __hip_atomic_store(&first[l], fz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&count[l], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();
  __syncthreads();
  for (int j = tid; j < fz; j += nt) {
    const DevPlane p = dev_classify(z_begin, z_end, fz, L, d, j);
    if (p.kind == 1) {
      atomicMin(&first[p.layer], j);
      atomicAdd(&count[p.layer], 1);
    }
  }
  __threadfence();
  __syncthreads();
  const int chunk = (fz + nt - 1) / nt;
  const int j0 = min(fz, tid * chunk), j1 = min(fz, j0 + chunk);
  int n_task = 0, n_ext = 0;
  for (int j = j0; j < j1; ++j) {
    const DevPlane p = dev_classify(z_begin, z_end, fz, L, d, j);
    if (p.kind != 1)
      ++n_ext;
    else if ((j - load_agent(&first[p.layer])) % zt == 0)
      ++n_task;
  }
  s_task[tid] = n_task;
  s_ext[tid] = n_ext;
  __syncthreads();
  if (tid == 0) {
    int a = 0, b = 0;
    for (int i = 0; i < nt; ++i) {
      const int x = s_task[i], y = s_ext[i];
      s_task[i] = a;
      s_ext[i] = b;
      a += x;
      b += y;
    }
  }
  __syncthreads();
  int ti = s_task[tid], ei = s_ext[tid];
  for (int j = j0; j < j1; ++j) {
    const DevPlane p = dev_classify(z_begin, z_end, fz, L, d, j);
    if (p.kind != 1) {
      if (ei < n_ext_max) ext[ei] = ExtPlane{j, p.kind, p.dz_top};
      ++ei;
      continue;
    }
    const int r = j - load_agent(&first[p.layer]);
    if (r % zt || ti >= ntasks) continue;  // the host sized the tables with the same rule
    const int cnt = min(zt, load_agent(&count[p.layer]) - r);
    tasks[ti] = Task{p.layer, j, cnt, 0};
    for (int q = 0; q < zt; ++q) {
      double top = 0.0, bot = 0.0;
      if (q < cnt) {
        const DevPlane pq = dev_classify(z_begin, z_end, fz, L, d, j + q);
        top = pq.dz_top;
        bot = pq.dz_bot;
      }
      const size_t o = ((size_t)ti * zt + q) * 2;
      task_dz[o] = top;
      task_dz[o + 1] = bot;
      task_dz32[o] = (float)top;
      task_dz32[o + 1] = (float)bot;
    }
    ++ti;
  }
}

// e^{2 pi i idx / n} with idx reduced modulo n in integers.
__device__ double2 dev_twiddle(long long idx, int n) {
  long long r = idx % n;
  if (r < 0) r += n;
  const double ang = __ddiv_rn(__dmul_rn(2.0 * M_PI, (double)r), (double)n);
  double sn, cs;
  sincos(ang, &sn, &cs);
  return make_double2(cs, sn);
}

// twx [2][fx], twy [2][fy] and, when R > 0, the factored transform's [R][32].
template <typename T>
__global__ void noalloc_twiddles_kernel(int fx, int fy, int U, int V, int R, T* __restrict__ twx,
                                        T* __restrict__ twy, T* __restrict__ fft_tw) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nx = 2LL * fx, ny = 2LL * fy, nr = 32LL * R;
  double2 w;
  T* out;
  if (i < nx) {
    const long long f = i < fx ? i : i - fx;
    w = dev_twiddle(i < fx ? f : -(long long)(U / 2) * f, fx);
    out = twx + 2 * i;
  } else if (i < nx + ny) {
    const long long k = i - nx;
    const long long g = k < fy ? k : k - fy;
    w = dev_twiddle(k < fy ? g : -(long long)(V / 2) * g, fy);
    out = twy + 2 * k;
  } else if (i < nx + ny + nr) {
    const long long k = i - nx - ny;
    const long long g1 = k / 32, sl = k % 32;
    w = dev_twiddle((sl - 16) * g1, fy);
    out = fft_tw + 2 * k;
  } else {
    return;
  }
  out[0] = (T)w.x;
  out[1] = (T)w.y;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

int noalloc_attach(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SCW_EINVAL, "device index " + std::to_string(device) + " beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_attach_lock);
  if (g_scratch_ptr[device]) return SCW_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(SCW_EHIP, std::string("hipGetSymbolAddress of the scratch array: ") +
                              hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return SCW_OK;
}

}  // namespace scw

using namespace scw;

extern "C" int scw_synthesize_noalloc(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid,
                                      int precision, void* E_dev, void* hip_stream) {
  if (!ctx || !sol || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision != SCW_FP64 && precision != SCW_FP32)
    return fail(SCW_EINVAL, "the allocation-free synthesis takes SCW_FP64 or SCW_FP32");
  Context& c = ctx->c;
  Solution& s = sol->s;
  if (s.device != c.device) return fail(SCW_EINVAL, "solution belongs to another device");
  if (precision == SCW_FP32 && !s.d_P32.p)
    return fail(SCW_EINVAL, "solution has no FP32 synthesis matrices");
  void* base = (c.device >= 0 && c.device < kMaxDevices) ? g_scratch_ptr[c.device] : nullptr;
  if (!base) return fail(SCW_EHIP, "scratch array not attached on this device");
  const scw_grid& g = *grid;
  const PlaneGroups pg = plane_group_shape(g, s.L, s.d);
  scw_synth_config cfg = resolve_config(c, s, g, precision);
  KernelShape ks{};
  if ((rc = choose_shape(s, g, precision, cfg, pg.zt, &ks))) return rc;
  if (ks.kind == SCW_XFORM_MFMA) {  // its operands are host-built: factored or direct instead
    cfg.transform = ks.fft_ok ? SCW_XFORM_FFT : SCW_XFORM_DIRECT;
    cfg.tiles = 0;
    if ((rc = choose_shape(s, g, precision, cfg, pg.zt, &ks))) return rc;
  }
  const size_t eb = precision == SCW_FP64 ? 16 : 8;
  const size_t n2 = 2 * (size_t)s.M;
  const int R = ks.fft_p > 0 ? g.fy / ks.fft_p : 0;
  // layout of the scratch array, every region 256-byte aligned
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 16));
    return o;
  };
  const size_t o_first = take((size_t)s.L * 4), o_count = take((size_t)s.L * 4);
  const size_t o_tasks = take((size_t)pg.ntasks * sizeof(Task));
  const size_t o_dz = take((size_t)pg.ntasks * pg.zt * 2 * sizeof(double));
  const size_t o_dz32 = take((size_t)pg.ntasks * pg.zt * 2 * sizeof(float));
  const size_t o_ext = take((size_t)pg.n_ext * sizeof(ExtPlane));
  const size_t o_w = take(precision == SCW_FP64 ? (size_t)pg.ntasks * 2 * pg.zt * n2 * eb : 0);
  const size_t o_spec = take((size_t)g.fz * 3 * s.M * eb);
  const size_t o_twx = take(2 * (size_t)g.fx * eb), o_twy = take(2 * (size_t)g.fy * eb);
  const size_t o_fft = take(32 * (size_t)R * eb);
  if (off > SCW_NOALLOC_SCRATCH_BYTES)
    return fail(SCW_EINVAL, "allocation-free synthesis needs " + std::to_string(off) +
                                " bytes of scratch, above its limit of " +
                                std::to_string((size_t)SCW_NOALLOC_SCRATCH_BYTES));
  char* b = static_cast<char*>(base);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  SCW_HIP(hipSetDevice(c.device));
  noalloc_planes_kernel<<<1, 1024, 0, st>>>(
      g.z_begin, g.z_end, g.fz, s.L, s.d, pg.zt, pg.ntasks, pg.n_ext,
      reinterpret_cast<int*>(b + o_first),
      reinterpret_cast<int*>(b + o_count), reinterpret_cast<Task*>(b + o_tasks),
      reinterpret_cast<double*>(b + o_dz), reinterpret_cast<float*>(b + o_dz32),
      reinterpret_cast<ExtPlane*>(b + o_ext));
  SCW_HIP(hipGetLastError());
  const long long ntw = 2LL * g.fx + 2LL * g.fy + 32LL * R;
  const unsigned tw_blocks = (unsigned)((ntw + 255) / 256);
  if (precision == SCW_FP64)
    noalloc_twiddles_kernel<double><<<tw_blocks, 256, 0, st>>>(
        g.fx, g.fy, s.U, s.V, R, reinterpret_cast<double*>(b + o_twx),
        reinterpret_cast<double*>(b + o_twy), reinterpret_cast<double*>(b + o_fft));
  else
    noalloc_twiddles_kernel<float><<<tw_blocks, 256, 0, st>>>(
        g.fx, g.fy, s.U, s.V, R, reinterpret_cast<float*>(b + o_twx),
        reinterpret_cast<float*>(b + o_twy), reinterpret_cast<float*>(b + o_fft));
  SCW_HIP(hipGetLastError());
  SynthArgs a{};
  a.M = s.M;
  a.U = s.U;
  a.V = s.V;
  a.L = s.L;
  a.fx = g.fx;
  a.fy = g.fy;
  a.fz = g.fz;
  a.zt = pg.zt;
  a.ntasks = pg.ntasks;
  a.n_ext = pg.n_ext;
  a.P = precision == SCW_FP64 ? s.d_P64.p : s.d_P32.p;
  a.kg = s.d_kg.as<double>();
  a.a = s.d_a.as<double>();
  a.b = s.d_b.as<double>();
  a.ext = s.d_ext.as<double>();
  a.ksz = s.d_ksz.as<double>();
  a.tasks = reinterpret_cast<const Task*>(b + o_tasks);
  a.task_dz = reinterpret_cast<const double*>(b + o_dz);
  a.ext_planes = b + o_ext;
  a.w = b + o_w;
  a.spec = b + o_spec;
  a.twx = b + o_twx;
  a.twy = b + o_twy;
  a.E = E_dev;
  a.kgab32 = s.d_kgab32.p;
  a.task_dz32 = b + o_dz32;
  a.precision = precision;
  a.mfma = false;
  a.kp = 0;
  a.fft_p = ks.fft_p;
  a.fft_tw = b + o_fft;
  a.idft_gtiles = ks.tiles;
  a.modal_rw = ks.modal_rw;
  a.stages = kStageAll;
  SCW_HIP(precision == SCW_FP64 ? launch_synthesis_fp64(a, st, nullptr)
                                : launch_synthesis_fp32(a, st, nullptr));
  return SCW_OK;
}
