// Dry run of whole solves through the C ABI with the host-only HIP stand-in
// (hip_mock.cpp): every launch the engine issues is audited instead of run.
//
// usage: dryrun <psf-file> <m> <levels> <solver> <wavelet> <transfer> <precision>
//               <k_out> <k_in> <small_cgls> <copies> [<inner> [<gcv mode>]]
// psf-file: "ph pw" then ph*pw values, column-major; a comma-separated list
// of such files gives the copies their PSFs in turn.  copies > 1 solves that
// many copies of the request in one dbl_deblur_batch call.
// DRYRUN_MULTI_TILES sets DBL_OPT_MULTI_BUCKET.  Parameters are a
// fixed schedule, or chosen by GCV when a GCV mode is given (the stand-in's
// device memory holds zeros, so the minimisations run their full length).  Prints the launch counts per kernel family and
// every violation; exits 1 when there is one.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/deblur.h"

namespace mock {
extern std::vector<std::string> violations;
extern std::map<std::string, long> launches;
extern long checked_pointers;
extern std::map<std::string, long> copies_before;
}  // namespace mock

int main(int argc, char** argv) {
  if (argc < 12) {
    std::fprintf(stderr, "usage: dryrun psf m levels solver wavelet transfer precision k_out k_in "
                         "small copies [inner]\n");
    return 2;
  }
  struct Psf {
    int ph = 0, pw = 0;
    std::vector<double> v;
  };
  std::vector<Psf> psfs;
  {
    std::string list = argv[1];
    size_t at = 0;
    while (at <= list.size()) {
      const size_t cut = std::min(list.find(',', at), list.size());
      FILE* f = std::fopen(list.substr(at, cut - at).c_str(), "r");
      if (!f) return 2;
      Psf p;
      if (std::fscanf(f, "%d %d", &p.ph, &p.pw) != 2) return 2;
      p.v.resize((size_t)p.ph * p.pw);
      for (double& v : p.v)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
      std::fclose(f);
      psfs.push_back(std::move(p));
      at = cut + 1;
    }
  }
  const int ph = psfs[0].ph, pw = psfs[0].pw;
  std::vector<double>& psf = psfs[0].v;
  const int m = std::atoi(argv[2]), levels = std::atoi(argv[3]), solver = std::atoi(argv[4]),
            wavelet = std::atoi(argv[5]), transfer = std::atoi(argv[6]),
            prec = std::atoi(argv[7]), k_out = std::atoi(argv[8]), k_in = std::atoi(argv[9]),
            small = std::atoi(argv[10]), copies = std::atoi(argv[11]);
  const int inner = argc > 12 ? std::atoi(argv[12]) : DBL_INNER_CGLS;
  const int gcv = argc > 13 ? std::atoi(argv[13]) : 0;  // 0: fixed parameters; else a GCV mode

  dbl_ctx* ctx = nullptr;
  int rc = dbl_create(&ctx, 0, nullptr, 0);
  if (rc) return 3;
  dbl_set_option(ctx, DBL_OPT_SMALL_CGLS, small);
  if (const char* mt = std::getenv("DRYRUN_MULTI_TILES"))
    dbl_set_option(ctx, DBL_OPT_MULTI_BUCKET, std::atoll(mt));
  if (std::getenv("DRYRUN_AUTOTUNE")) {
    // the tuner's synthetic launches are audited like the solve's; the
    // stand-in's events read 0 ms, so every key keeps variant 0
    int n = 0;
    rc = dbl_autotune(ctx, prec, nullptr, DBL_TUNE_QUICK, &n);
    std::printf("autotune status %d entries %d\n", rc, n);
    if (rc) return 1;
  }
  const size_t esz = prec == DBL_F64 ? 8 : 4;
  std::vector<double> mu((size_t)levels * k_out);
  for (int i = 0; i < levels; ++i)
    for (int k = 0; k < k_out; ++k) mu[(size_t)i * k_out + k] = 1e-3 * (1 << i);
  dbl_opts o;
  dbl_opts_default(&o);
  o.k_out = k_out;
  o.k_in = k_in;
  o.precision = prec;
  o.mu_schedule = gcv ? nullptr : mu.data();
  if (gcv) o.gcv_mode = gcv;
  o.inner_solver = inner;
  std::vector<dbl_request> reqs(copies);
  for (int q = 0; q < copies; ++q) {
    void *b = nullptr, *x = nullptr;
    hipMalloc(&b, (size_t)m * m * esz);
    // DRYRUN_SHORT_X: an x buffer one element too short (the audit must see it)
    hipMalloc(&x, ((size_t)m * m - (std::getenv("DRYRUN_SHORT_X") ? 1 : 0)) * esz);
    const Psf& p = psfs[q % psfs.size()];
    reqs[q] = dbl_request{b, x, p.v.data(), p.ph, p.pw, m, solver, wavelet, levels, transfer, o};
  }
  dbl_report rep;
  if (copies == 1)
    rc = dbl_deblur(ctx, reqs[0].b, psf.data(), ph, pw, m, solver, wavelet, levels, transfer, &o,
                    reqs[0].x, &rep);
  else
    rc = dbl_deblur_batch(ctx, copies, reqs.data(), nullptr);
  std::printf("status %d (%s)\n", rc, rc ? dbl_last_error(ctx) : "ok");
  for (auto& kv : mock::launches) std::printf("launches %s %ld\n", kv.first.c_str(), kv.second);
  long n_copies = 0;
  for (auto& kv : mock::copies_before) {
    if (kv.second) std::printf("copies before %s %ld\n", kv.first.c_str(), kv.second);
    n_copies += kv.second;
  }
  std::printf("copies %ld\n", n_copies);
  std::printf("checked %ld pointers\n", mock::checked_pointers);
  for (auto& v : mock::violations) std::printf("VIOLATION %s\n", v.c_str());
  std::printf("violations %zu\n", mock::violations.size());
  dbl_destroy(ctx);
  return (rc || !mock::violations.empty()) ? 1 : 0;
}
