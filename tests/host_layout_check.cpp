// CPU driver for the library's host-side logic (host_layout.h), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
// It sweeps grid shapes, precisions, walls, densities, record lengths and the
// launch-shape overrides, and checks that every launch covers its grid, that
// the workspace regions are aligned, ordered and large enough, that the
// checkpoint spacing is ceil(sqrt(N)), and that invalid parameters are
// refused with a reason.  Prints "ok <cases>" and exits 0 when all hold.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "host_layout.h"

using namespace lbe;
using namespace lbe::host;

static int g_fail = 0;
#define CHECK(cond, ...)                                                     \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "FAIL %s:%d %s: ", __FILE__, __LINE__, #cond);    \
      std::fprintf(stderr, __VA_ARGS__);                                     \
      std::fprintf(stderr, "\n");                                            \
      if (++g_fail > 20) std::exit(1);                                       \
    }                                                                        \
  } while (0)

static lbe_csf_params base(int nx, int ny) {
  lbe_csf_params p{};
  p.nx = nx;
  p.ny = ny;
  p.walls_y = 1;
  p.precision = LBE_CSF_FP32_DEV;
  p.rho = p.cv = 1.0;
  p.tau_f[0] = p.tau_f[1] = 0.8;
  p.tau_T[0] = p.tau_T[1] = 0.7;
  p.tau_g = 1.0;
  p.mobility = 0.05;
  p.width = 2.8284271247461903;
  p.beta = 0.25;
  p.sigma0 = 1e-2;
  p.sigmaT = 5e-4;
  p.T_grad = 0.01;
  return p;
}

static void check_launch(const Launch &L, int nx, int ny, bool two) {
  CHECK(L.nw == 1 || L.nw == 2 || L.nw == 4 || L.nw == 8, "nw %d", L.nw);
  const long bx = 64L * L.nw;
  CHECK(L.nstrips * bx >= nx && (L.nstrips - 1) * bx < nx, "strips %d x %ld for nx %d",
        L.nstrips, bx, nx);
  CHECK(L.rows >= 1 && L.rows <= ny, "rows %d ny %d", L.rows, ny);
  CHECK((long)L.nchunks * L.rows >= ny && (long)(L.nchunks - 1) * L.rows < ny,
        "chunks %d x %d for ny %d", L.nchunks, L.rows, ny);
  CHECK(L.nblocks == L.nstrips * L.nchunks, "nblocks %d", L.nblocks);
  CHECK(L.pipe >= 0 && L.pipe <= 2, "pipe %d", L.pipe);
  if (two) CHECK(L.pipe == 1, "two densities need rows one ahead (pipe %d)", L.pipe);
}

static void check_layout(const lbe_csf_params &p, int64_t rec) {
  const Layout L = make_layout(&p, rec);
  const size_t n = (size_t)p.nx * p.ny;
  const bool f64 = p.precision == LBE_CSF_FP64;
  const size_t sb = f64 ? state_bytes_for<double>(n) : state_bytes_for<float>(n);
  CHECK(L.state_bytes == sb, "state bytes");
  // row-interleaved state: ny rows of row_bytes, each 25 plane segments then
  // g_0 and hbar_0; every byte offset a kernel forms fits its 32-bit offset
  const size_t rb = f64 ? row_bytes<double>(p.nx) : row_bytes<float>(p.nx);
  const size_t vb = f64 ? 8 : 4;
  CHECK(rb * p.ny == sb, "rows x row bytes");
  const size_t r0 = f64 ? rest_base<double>(0, p.nx) : rest_base<float>(0, p.nx);
  const size_t r1 = f64 ? rest_base<double>(1, p.nx) : rest_base<float>(1, p.nx);
  CHECK(r0 == kNumS * p.nx * vb, "g_0 after the 25 plane segments");
  CHECK(r1 == r0 + (size_t)p.nx * 8, "hbar_0 after g_0 (FP64)");
  CHECK(r1 + (size_t)p.nx * vb == rb, "hbar_0 ends the row");
  CHECK(sb - 1 <= 0xffffffffull, "state offsets fit 32 bits");
  const Launch la = pick_launch(p.nx, p.ny, !f64, !two_densities(&p));
  check_launch(la, p.nx, p.ny, two_densities(&p));
  // one density or FP64, wide enough for a full strip and tall enough for
  // chunks of four rows at one block per CU: that shape
  {
    const int nw1 = f64 ? 4 : 8;
    const int nstr = (p.nx + 64 * nw1 - 1) / (64 * nw1);
    const int chunks = std::max(1, kNumCUs / nstr);
    const bool env = std::getenv("LBE_CSF_NW") || std::getenv("LBE_CSF_ROWS") ||
                     std::getenv("LBE_CSF_PIPE");
    if (!env && (!two_densities(&p) || f64) && p.nx >= 64 * nw1 &&
        (p.ny + chunks - 1) / chunks >= 4)
      CHECK(la.nw == nw1 && la.nblocks <= kNumCUs && la.pipe == (f64 ? 1 : 2),
            "one block per CU (nw %d, %d blocks, pipe %d)", la.nw, la.nblocks, la.pipe);
  }
  // the store policy: whole-line stores bypass the last-level cache for the
  // FP32 one-density step whose two states exceed it
  const Launch lf = launch_for(&p, L.state_bytes);
  CHECK(lf.nblocks == la.nblocks && lf.pipe == la.pipe, "launch_for shape");
  CHECK(lf.stream == (!f64 && !two_densities(&p) && 2 * sb > kLastLevelCache), "store policy");
  // the small-grid path: only one density, at most one site per lane of a
  // 512-lane block, and the LDS of the padded moment grid (16-byte rounded);
  // with the states resident, both states after it
  const size_t sl = small_lds_bytes(&p), sr = small_res_bytes(&p);
  if (two_densities(&p) || n > (size_t)kSmallMaxSites) {
    CHECK(sl == 0 && sr == 0, "small path on %dx%d", p.nx, p.ny);
  } else {
    const size_t m = (size_t)(p.nx + 2) * (p.ny + 2) * (f64 ? 24 : 16);
    CHECK(sl >= m && sl < m + 16 && sl % 16 == 0, "small LDS bytes");
    CHECK(sr == sl + 2 * sb, "resident small LDS bytes");
  }
  const size_t offs[] = {L.off_a, L.off_b, L.off_tw, L.off_part, L.off_ring,
                         L.off_cnt, L.off_rec, L.off_pc, L.off_adj};
  for (size_t o : offs) CHECK(o % kAlign == 0, "offset %zu not aligned", o);
  CHECK(L.off_b >= L.off_a + sb && L.off_tw >= L.off_b + sb, "states overlap");
  CHECK(L.off_part >= L.off_tw + 2 * (size_t)p.nx * 8, "wall region");
  CHECK(L.off_ring >= L.off_part + (size_t)la.nblocks * kNumPartials * 8, "partials region");
  CHECK(L.off_cnt >= L.off_ring + (size_t)kDiagRing * sizeof(DiagRecord), "ring region");
  CHECK(L.off_rec >= L.off_cnt + 4 * sizeof(int64_t), "counters");
  CHECK(L.off_pc >= L.off_rec + sizeof(DiagRecord), "record");
  CHECK(L.off_adj >= L.off_pc + (two_densities(&p) ? n * 8 : 0), "pressure plane");
  CHECK(L.total >= L.off_adj + L.adj.total, "total");
  if (rec > 0) {
    const AdjLayout &A = L.adj;
    CHECK(A.K * A.K >= rec && (rec <= 1 || (A.K - 1) * (A.K - 1) < rec), "K %lld for N %lld",
          (long long)A.K, (long long)rec);
    CHECK(A.nchk * A.K >= rec && (A.nchk - 1) * A.K < rec, "checkpoints");
    CHECK(A.state_bytes >= sb && A.state_bytes % 256 == 0, "checkpoint state size");
    CHECK(A.off_tape >= A.off_chk + (size_t)A.nchk * A.state_bytes, "checkpoint region");
    CHECK(A.off_tape2 >= A.off_tape + (size_t)A.K * (A.state_bytes + A.mom_bytes), "tape");
    CHECK(A.off_lam >= A.off_tape2 + 2 * A.state_bytes + (size_t)A.K * A.mom_bytes,
          "second tape");
    CHECK(A.off_part >= A.off_lam + (2 * 27 + 2 * 3 + kAdjA) * A.plane_bytes, "cotangents");
    CHECK(A.off_tw >= A.off_part + (size_t)adj_tiles_x(p.nx) * adj_tiles_y(p.ny) * 8, "adj part");
    CHECK(A.total >= A.off_tw + 2 * (size_t)p.nx * 8 + 8, "adj total");
  } else {
    CHECK(L.adj.total == 0, "no adjoint region without a record");
  }
}

int main() {
  const int sizes[] = {3, 4, 5, 7, 8, 9, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257,
                       511, 512, 513, 1000, 2047, 2048, 4095, 4096, 5000, 8192};
  const int64_t recs[] = {0, 1, 2, 7, 64, 4000};
  long cases = 0;
  for (const char *nw : {"", "1", "2", "4", "8"})
    for (const char *rows : {"", "1", "3", "64"})
      for (const char *pipe : {"", "0", "2"}) {
        if (*nw) setenv("LBE_CSF_NW", nw, 1); else unsetenv("LBE_CSF_NW");
        if (*rows) setenv("LBE_CSF_ROWS", rows, 1); else unsetenv("LBE_CSF_ROWS");
        if (*pipe) setenv("LBE_CSF_PIPE", pipe, 1); else unsetenv("LBE_CSF_PIPE");
        for (int nx : sizes)
          for (int ny : sizes)
            for (int prec : {LBE_CSF_FP64, LBE_CSF_FP32_DEV})
              for (double rho2 : {0.0, 2.0}) {
                lbe_csf_params p = base(nx, ny);
                p.precision = prec;
                p.rho2 = rho2;
                std::string why;
                const bool ok = params_valid(&p, &why);
                const size_t n = (size_t)nx * ny;
                const double sb = prec == LBE_CSF_FP64 ? (double)state_bytes_for<double>(n)
                                                       : (double)state_bytes_for<float>(n);
                CHECK(ok == (sb < 4294967296.0), "%dx%d prec %d: %s", nx, ny, prec, why.c_str());
                if (!ok) {
                  CHECK(!why.empty(), "refusal without a reason");
                  continue;
                }
                for (int64_t rec : recs) {
                  if (rec > 0 && (size_t)n * rec > (size_t)1 << 31) continue;
                  check_layout(p, rec);
                  ++cases;
                }
              }
      }
  unsetenv("LBE_CSF_NW");
  unsetenv("LBE_CSF_ROWS");
  unsetenv("LBE_CSF_PIPE");
  // invalid parameters are refused with a reason
  struct Bad {
    const char *what;
    void (*set)(lbe_csf_params &);
  };
  const Bad bad[] = {
      {"nx", [](lbe_csf_params &p) { p.nx = 2; }},
      {"ny", [](lbe_csf_params &p) { p.ny = -5; }},
      {"tau_f", [](lbe_csf_params &p) { p.tau_f[1] = 0.5; }},
      {"tau_T", [](lbe_csf_params &p) { p.tau_T[0] = 0.3; }},
      {"tau_g", [](lbe_csf_params &p) { p.tau_g = 0.5; }},
      {"mobility", [](lbe_csf_params &p) { p.mobility = 0.0; }},
      {"width", [](lbe_csf_params &p) { p.width = -1.0; }},
      {"beta", [](lbe_csf_params &p) { p.beta = 0.0; }},
      {"rho", [](lbe_csf_params &p) { p.rho = 0.0; }},
      {"walls", [](lbe_csf_params &p) { p.walls_y = 2; }},
      {"precision", [](lbe_csf_params &p) { p.precision = 7; }},
      {"csf_form", [](lbe_csf_params &p) { p.csf_form = 3; }},
      {"rho2", [](lbe_csf_params &p) { p.rho2 = -1.0; }},
      {"sigmaT", [](lbe_csf_params &p) { p.sigmaT = std::nan(""); }},
      {"T_grad periodic", [](lbe_csf_params &p) { p.walls_y = 0; }},
      {"diag_every", [](lbe_csf_params &p) { p.diag_every = -1; }},
  };
  for (const Bad &b : bad) {
    lbe_csf_params p = base(64, 64);
    b.set(p);
    std::string why;
    CHECK(!params_valid(&p, &why) && !why.empty(), "%s accepted", b.what);
  }
  CHECK(!params_valid(nullptr, nullptr), "NULL params accepted");
  // the step kernel chosen at measured points (tiles or row-marching chunks)
  unsetenv("LBE_CSF_TILE");
  struct TileCase {
    int nx, ny, prec;
    bool tile;
  };
  const TileCase tiles[] = {
      {16, 32, LBE_CSF_FP32_DEV, false},    {40, 100, LBE_CSF_FP32_DEV, true},
      {200, 100, LBE_CSF_FP32_DEV, true},  {200, 100, LBE_CSF_FP64, true},
      {201, 100, LBE_CSF_FP32_DEV, true},   {200, 1000, LBE_CSF_FP32_DEV, true},
      {70, 100, LBE_CSF_FP64, true},       {70, 100, LBE_CSF_FP32_DEV, true},
      {68, 400, LBE_CSF_FP64, true},        {70, 1000, LBE_CSF_FP32_DEV, true},
      {130, 100, LBE_CSF_FP32_DEV, true},   {520, 100, LBE_CSF_FP32_DEV, true},
      {1024, 1024, LBE_CSF_FP32_DEV, true}, {1024, 1024, LBE_CSF_FP64, false},
      {2048, 1024, LBE_CSF_FP32_DEV, false}, {1500, 700, LBE_CSF_FP32_DEV, true},
      {1500, 1500, LBE_CSF_FP32_DEV, false}, {1030, 1000, LBE_CSF_FP64, true},
      {800, 800, LBE_CSF_FP64, true},       {2048, 512, LBE_CSF_FP64, false},
      {2048, 1024, LBE_CSF_FP64, false},    {4096, 4096, LBE_CSF_FP32_DEV, false}};
  for (const TileCase &t : tiles) {
    lbe_csf_params p = base(t.nx, t.ny);
    p.precision = t.prec;
    CHECK(use_tile_kernel(&p) == t.tile, "%dx%d prec %d: tile kernel %d expected", t.nx, t.ny,
          t.prec, (int)t.tile);
  }
  if (g_fail) return 1;
  std::printf("ok %ld\n", cases);
  return 0;
}
