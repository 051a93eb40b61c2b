// Host set-up under AddressSanitizer and UndefinedBehaviorSanitizer: reads
// cases (parameters, mesh, initial state) from a binary file and runs the
// library's host half of dg_create on each (parameter checks, workspace
// layout, bases, curl-form metrics, face checks, connectivity) and the host
// time-step estimate.  None of it calls HIP, so it runs on any CPU.
//
// Case file, native byte order, repeated until a zero flag:
//   int32 flag (1), dg_params, int64 n_elems, int32 n_geo,
//   double x_geo[E][3][(n_geo+1)^3], int64 nbr_elem[E][6],
//   int8 nbr_face[E][6], int8 nbr_orient[E][6], int64 count, double U0[count]
// (count is 5 E (N+1)^3 for a consistent case)
// Output, one line per case: "case <k> rc <status> dt <dt> bytes <layout> err <message>"
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dgsem.h"
#include "solver_impl.h"

template <typename T>
static bool take(FILE *f, T *dst, size_t count) {
  return count == 0 || std::fread(dst, sizeof(T), count, f) == count;
}

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s cases.bin\n", argv[0]);
    return 2;
  }
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  for (int k = 0;; ++k) {
    int32_t flag = 0;
    if (!take(f, &flag, 1) || flag == 0) break;
    dg_params p;
    int64_t E = 0;
    int32_t ngeo = 0;
    if (!take(f, &p, 1) || !take(f, &E, 1) || !take(f, &ngeo, 1)) return 3;
    const size_t ng = (size_t)ngeo + 1;
    // exact-size host copies, so that any read past an array is caught
    std::vector<double> x((size_t)E * 3 * ng * ng * ng);
    std::vector<int64_t> ne((size_t)E * 6);
    std::vector<int8_t> nf((size_t)E * 6), no((size_t)E * 6);
    int64_t count = 0;
    if (!take(f, x.data(), x.size()) || !take(f, ne.data(), ne.size()) || !take(f, nf.data(), nf.size()) ||
        !take(f, no.data(), no.size()) || !take(f, &count, 1))
      return 3;
    std::vector<double> U((size_t)count);
    if (!take(f, U.data(), U.size())) return 3;
    dg_mesh m{};
    m.n_elems = E;
    m.n_geo = ngeo;
    m.x_geo = x.data();
    m.nbr_elem = ne.data();
    m.nbr_face = nf.data();
    m.nbr_orient = no.data();
    std::string err;
    double dt = 0.0;
    size_t bytes = 0;
    // the checks dg_create makes before the host set-up
    dg_status rc = dg::check_params(&p);
    if (rc) err = dg_last_error();
    if (rc == DG_OK && (!dg::elems_in_range(p.N, E) || ngeo < 1 || ngeo > p.N)) {
      rc = DG_EINVAL;
      err = "mesh size or geometry degree out of range";
    }
    const int64_t n = p.N + 1;
    if (rc == DG_OK && count != 5 * E * n * n * n) {
      rc = DG_EINVAL;
      err = "state size does not match the mesh";
    }
    if (rc == DG_OK) {
      bytes = dg::make_layout(p, E).total;
      dg::HostSetup hs;
      rc = dg::setup_host(p, m, hs, err);
      if (rc == DG_OK) dt = dg::host_stable_dt(p, E, hs, U.data(), 0.9);
    }
    for (char &c : err)
      if (c == '\n') c = ' ';
    std::printf("case %d rc %d dt %.17g bytes %zu err %s\n", k, (int)rc, dt, bytes, err.c_str());
  }
  std::fclose(f);
  return 0;
}
