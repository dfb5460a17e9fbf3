// Host-side lifetime and memory check of libpic's C ABI (test infrastructure).  Built with the
// library's own sources compiled for the host only, linked against hip_stub.cpp (a stand-in
// HIP runtime that checks handle lifetimes and capture joins) and run under AddressSanitizer.
//
// It drives the create / track / destroy sequences of the GPU test suite in the order the
// Python binding runs them, above all the one that once ended in a host segmentation fault:
// two batches of beams created one after the other, the first batch and its beams destroyed
// (Python rebinding: new beams and batch created first, then the old batch, then the old
// beams) before the second batch's first pic_track_batch, which captures its graph.  It also
// destroys batches and beams right after enqueuing work, without a synchronisation, which the
// library must make safe.  Exit status 0 and no ASan report: every sequence is clean.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pic.h"

extern "C" long long hip_stub_launch_count();
extern "C" int hip_stub_live_handles();
extern "C" int hipStreamCreateWithFlags(void** s, unsigned int flags);
extern "C" int hipStreamDestroy(void* s);
extern "C" int hipStreamSynchronize(void* s);

namespace {

int g_fail = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "lifetimes: FAILED %s: %s\n", what, pic_last_error());
    ++g_fail;
  }
}

// a beam whose "device" arrays are zeroed host memory
struct HostBeam {
  pic_beam h = nullptr;
  std::vector<double> X;
  void* work = nullptr;
  void* rho = nullptr;
  void* E = nullptr;
  void* Ep = nullptr;
  int64_t n = 0;
};

pic_beam_desc desc(int64_t n, int nx, int ny, int nz, int shape, int fp32 = 0, int direct = 0) {
  pic_beam_desc d;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.qm_qeeV = -1.0 / 0.51099895e6;
  d.charge_C = 1e-9;
  d.kin_energy_MeV = 20.0;
  d.mass_MeV = 0.51099895;
  d.shape = shape;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.grid_fp32 = fp32;
  d.space_charge = 1;
  d.direct_field = direct;
  return d;
}

void* zalloc(size_t bytes) {
  void* p = nullptr;
  if (posix_memalign(&p, 256, bytes ? bytes : 256) != 0) std::abort();
  std::memset(p, 0, bytes ? bytes : 256);
  return p;
}

HostBeam* make_beam(const pic_beam_desc& d, void* stream) {
  HostBeam* b = new HostBeam;
  b->n = d.n;
  b->X.assign(6 * (size_t)d.n, 0.0);
  const size_t wb = pic_workspace_bytes(&d);
  expect(wb > 0, "pic_workspace_bytes");
  b->work = zalloc(wb);
  const size_t es = d.grid_fp32 ? 4 : 8;
  const size_t ng = (size_t)d.nx * d.ny * d.nz;
  b->rho = zalloc(es * ng);
  b->E = zalloc(3 * es * ng);
  b->Ep = zalloc(3 * es * (size_t)d.n);
  expect(pic_beam_create(&d, b->X.data(), b->work, wb, stream, &b->h) == PIC_OK,
         "pic_beam_create");
  double sigma[36] = {0};
  const double diag[6] = {1e-6, 1e-6, 1e-6, 1e-6, 4e-6, 1e-6};
  for (int a = 0; a < 6; ++a) sigma[a * 6 + a] = diag[a];
  expect(pic_init_beam(b->h, sigma, 7, 0.1, stream) == PIC_OK, "pic_init_beam");
  return b;
}

void free_beam(HostBeam* b) {
  expect(pic_beam_destroy(b->h) == PIC_OK, "pic_beam_destroy");
  std::free(b->work);
  std::free(b->rho);
  std::free(b->E);
  std::free(b->Ep);
  delete b;
}

struct HostBatch {
  pic_batch h = nullptr;
  void* work = nullptr;
};

HostBatch* make_batch(const std::vector<HostBeam*>& beams,
                      const std::vector<std::vector<pic_element>>& lats, void* stream,
                      int expect_status = PIC_OK) {
  const int nb = (int)beams.size();
  std::vector<pic_beam> hs(nb);
  std::vector<const pic_element*> lp(nb);
  std::vector<int> ne(nb);
  for (int i = 0; i < nb; ++i) {
    hs[i] = beams[i]->h;
    lp[i] = lats[i].data();
    ne[i] = (int)lats[i].size();
  }
  const size_t wb = pic_batch_workspace_bytes(nb, lp.data(), ne.data());
  expect(wb > 0, "pic_batch_workspace_bytes");
  HostBatch* bt = new HostBatch;
  bt->work = zalloc(wb);
  const int st = pic_batch_create(hs.data(), nb, lp.data(), ne.data(), 0, bt->work, wb, stream,
                                  &bt->h);
  expect(st == expect_status, "pic_batch_create status");
  return bt;
}

void free_batch(HostBatch* bt) {
  if (bt->h) expect(pic_batch_destroy(bt->h) == PIC_OK, "pic_batch_destroy");
  std::free(bt->work);
  delete bt;
}

std::vector<pic_element> thin_fodo(double k) {
  pic_element a{}, c{};
  a.kind = PIC_ELEM_THIN;
  a.k = k;
  a.ds = 0.5;
  c = a;
  c.k = -k;
  return {a, c};
}

std::vector<pic_element> thick_cell() {
  std::vector<pic_element> v(5);
  const int kind[5] = {PIC_ELEM_DRIFT, PIC_ELEM_QUAD, PIC_ELEM_DRIFT, PIC_ELEM_QUAD,
                       PIC_ELEM_DRIFT};
  const double ds[5] = {0.25, 1.0, 0.5, 1.0, 0.25}, k[5] = {0, 1.0, 0, -1.0, 0};
  for (int i = 0; i < 5; ++i) {
    v[i].kind = kind[i];
    v[i].ds = ds[i];
    v[i].k = k[i];
    v[i].nslice = 3;
  }
  return v;
}

}  // namespace

int main() {
  void* s = nullptr;
  hipStreamCreateWithFlags(&s, 1);
  const int live0 = hip_stub_live_handles();

  // single-beam calls
  {
    HostBeam* b = make_beam(desc(4000, 16, 16, 16, 2), s);
    expect(pic_deposit(b->h, b->rho, s) == PIC_OK, "pic_deposit");
    expect(pic_poisson_solve(b->h, b->rho, nullptr, b->E, s) == PIC_OK, "pic_poisson_solve");
    expect(pic_gather(b->h, b->E, b->Ep, s) == PIC_OK, "pic_gather");
    expect(pic_push(b->h, PIC_PUSH_KICK, 0.5, b->Ep, s) == PIC_OK, "pic_push");
    auto lat = thin_fodo(1.0);
    expect(pic_profile_start(b->h) == PIC_OK, "pic_profile_start");
    expect(pic_track_n_steps(b->h, lat.data(), 2, 5, s) == PIC_OK, "pic_track_n_steps");
    double ms[8];
    int64_t cnt[8];
    expect(pic_profile_read(b->h, ms, cnt) == PIC_OK, "pic_profile_read");
    std::vector<double> diag(27 * 4);
    auto thick = thick_cell();
    expect(pic_track_n_steps_diag(b->h, thick.data(), 5, 4, diag.data(), s) == PIC_OK,
           "pic_track_n_steps_diag");
    double mean[6], cov[36], m4[4], geo[9];
    expect(pic_moments(b->h, mean, cov, s) == PIC_OK, "pic_moments");
    expect(pic_objective(b->h, m4, s) == PIC_OK, "pic_objective");
    expect(pic_get_geometry(b->h, geo, s) == PIC_OK, "pic_get_geometry");
    // reverse sweep
    const pic_beam_desc d = desc(4000, 16, 16, 16, 2);
    const size_t aw = pic_adjoint_workspace_bytes(&d, 6, 2);
    void* adj = zalloc(aw);
    std::vector<double> lam(6 * 4000), xi(6 * 4000, 0.0);
    const double w[4] = {1, 1, 1, 1};
    double dk[5], dL[36];
    expect(pic_track_adjoint(b->h, thick.data(), 5, 6, 2, w, adj, aw, lam.data(), xi.data(), m4,
                             dk, dL, s) == PIC_OK,
           "pic_track_adjoint");
    std::free(adj);
    // destroyed right after enqueuing a tracking call, with no synchronisation
    expect(pic_track_n_steps(b->h, lat.data(), 2, 3, s) == PIC_OK, "pic_track_n_steps");
    free_beam(b);
  }

  // the batch tests' beam mix, replayed; the rejection of the direct field
  {
    std::vector<HostBeam*> beams = {make_beam(desc(7001, 16, 16, 16, 1), s),
                                    make_beam(desc(12000, 24, 24, 24, 1), s),
                                    make_beam(desc(3000, 12, 18, 24, 1), s)};
    std::vector<std::vector<pic_element>> lats = {thin_fodo(1.0), thin_fodo(1.6), thick_cell()};
    HostBatch* bt = make_batch(beams, lats, s);
    expect(pic_track_batch(bt->h, 6, s) == PIC_OK, "pic_track_batch capture");
    expect(pic_track_batch(bt->h, 6, s) == PIC_OK, "pic_track_batch replay");
    expect(pic_track_batch(bt->h, 3, s) == PIC_OK, "pic_track_batch second graph");
    hipStreamSynchronize(s);
    free_batch(bt);
    for (HostBeam* b : beams) free_beam(b);
    HostBeam* df = make_beam(desc(2000, 16, 16, 16, 1, 0, 1), s);
    HostBatch* rej = make_batch({df}, {thin_fodo(1.0)}, s, PIC_EUNSUPPORTED);
    free_batch(rej);
    free_beam(df);
  }

  // the determinism test's loop: two batches one after the other, Python's teardown order
  {
    struct Mix {
      int64_t n;
      int nx, ny, nz;
      double k;
    } mix[3] = {{7001, 16, 16, 16, 1.0}, {12000, 24, 24, 24, 1.6}, {3000, 12, 18, 24, 0.7}};
    std::vector<HostBeam*> old_beams;
    HostBatch* old_batch = nullptr;
    for (int it = 0; it < 3; ++it) {
      std::vector<HostBeam*> beams;
      std::vector<std::vector<pic_element>> lats;
      for (const Mix& m : mix) {
        beams.push_back(make_beam(desc(m.n, m.nx, m.ny, m.nz, 2), s));
        lats.push_back(thin_fodo(m.k));
      }
      HostBatch* bt = make_batch(beams, lats, s);
      if (old_batch) free_batch(old_batch);
      for (HostBeam* b : old_beams) free_beam(b);
      expect(pic_track_batch(bt->h, 8, s) == PIC_OK, "pic_track_batch after teardown");
      if (it < 2) hipStreamSynchronize(s);  // the last batch is torn down unsynchronised
      old_batch = bt;
      old_beams = beams;
    }
    free_batch(old_batch);
    for (HostBeam* b : old_beams) free_beam(b);
  }

  hipStreamSynchronize(s);
  const int leaked = hip_stub_live_handles() - live0;
  expect(leaked == 0, "every stream, event and graph handle released");
  hipStreamDestroy(s);
  std::printf("lifetimes: %lld kernel launches, %d leaked handles, %d failures\n",
              hip_stub_launch_count(), leaked, g_fail);
  return g_fail ? 1 : 0;
}
