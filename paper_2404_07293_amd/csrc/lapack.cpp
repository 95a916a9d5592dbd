#include "lapack.h"

#include <dlfcn.h>
#include <stdlib.h>

#include <mutex>

namespace scw {

namespace {

Lapack g_lapack;
std::once_flag g_once;

template <typename F>
bool bind(void* h, const char* name, F& fn, std::string& err) {
  void* p = dlsym(h, name);
  if (!p) {
    err += std::string("missing symbol ") + name + "; ";
    return false;
  }
  fn = reinterpret_cast<F>(p);
  return true;
}

void load() {
  // MKL's threaded layer on GNU OpenMP, which is the OpenMP runtime the rest
  // of the process (PyTorch) already uses. A caller's own setting wins.
  setenv("MKL_THREADING_LAYER", "GNU", 0);
  const char* names[] = {"libmkl_rt.so.1", "libmkl_rt.so",
                         "/opt/conda/lib/libmkl_rt.so.1",
                         "/opt/conda/lib/libmkl_rt.so"};
  void* h = nullptr;
  const char* env = getenv("SCW_LAPACK_LIB");
  if (env && *env) h = dlopen(env, RTLD_NOW | RTLD_LOCAL);
  for (const char* n : names) {
    if (h) break;
    h = dlopen(n, RTLD_NOW | RTLD_LOCAL);
  }
  if (!h) {
    g_lapack.error = "could not load MKL (libmkl_rt.so.1); set SCW_LAPACK_LIB";
    return;
  }
  std::string err;
  bool ok = true;
  ok &= bind(h, "zgeev_", g_lapack.zgeev, err);
  ok &= bind(h, "zgetrf_", g_lapack.zgetrf, err);
  ok &= bind(h, "zgetrs_", g_lapack.zgetrs, err);
  ok &= bind(h, "zgemm_", g_lapack.zgemm, err);
  ok &= bind(h, "zgecon_", g_lapack.zgecon, err);
  ok &= bind(h, "zlange_", g_lapack.zlange, err);
  // C entry points (by-value int); the lower-case exports take a pointer.
  ok &= bind(h, "MKL_Set_Num_Threads_Local", g_lapack.set_threads_local, err);
  ok &= bind(h, "MKL_Set_Num_Threads", g_lapack.set_threads, err);
  g_lapack.ok = ok;
  g_lapack.error = err;
}

}  // namespace

const Lapack& lapack() {
  std::call_once(g_once, load);
  return g_lapack;
}

}  // namespace scw
