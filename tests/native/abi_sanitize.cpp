// Host-side checks of the C ABI layer under AddressSanitizer and UndefinedBehaviorSanitizer.
// Built from the library's host sources with -fsanitize on the host pass only (the kernels are
// the ordinary objects) and run on a machine without a GPU: every entry point is called with
// invalid arguments (each must return its error code without touching memory it was not
// given), and the calls that need a device are made with valid arguments so that their
// failure paths -- partial allocations released, no stream left behind -- run under the
// sanitizers.  Prints "OK" and exits 0 when every expectation holds.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ace.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++failures;
  }
}

int main() {
  // error strings for every code and a few out of range
  for (int code = -12; code <= 2; ++code) {
    const char* s = ace_strerror(code);
    expect(s != nullptr && std::strlen(s) > 0, "ace_strerror");
  }
  // compiled sizes
  int supported = 0;
  for (int n = -1; n <= 130; ++n)
    for (int dt = -1; dt <= 4; ++dt) supported += ace_size_supported(n, dt);
  expect(supported == 13 * 4, "ace_size_supported count");
  // trace class names
  for (int i = -1; i <= ace_trace_count(); ++i) (void)ace_trace_name(i);

  // contexts: argument checks
  ace_ctx* ctx = nullptr;
  expect(ace_ctx_create(16, 0.3, 9, nullptr, &ctx) == ACE_ERR_INVALID, "create bad dtype");
  expect(ace_ctx_create(11, 0.3, 0, nullptr, &ctx) == ACE_ERR_UNSUPPORTED, "create bad edge");
  expect(ace_ctx_create(16, -1.0, 0, nullptr, &ctx) == ACE_ERR_INVALID, "create bad h");
  expect(ace_ctx_create(16, 0.3, 0, nullptr, nullptr) == ACE_ERR_INVALID, "create null out");
  expect(ace_ctx_destroy(nullptr) == ACE_OK, "destroy null");
  expect(ace_ctx_set_stream(nullptr, nullptr) == ACE_ERR_INVALID, "set_stream null");
  int st = 0, info = 0;
  expect(ace_ctx_status(nullptr, &st, &info) == ACE_ERR_INVALID, "status null");

  // every compute entry point with a null context
  double d = 0.0;
  const int32_t pairs[2] = {0, 0};
  expect(pair_poisson_batched(nullptr, &d, 1, &d, 1, pairs, 1, &d) == ACE_ERR_INVALID, "pp");
  expect(pair_poisson_batched_dev(nullptr, &d, 1, &d, 1, pairs, 1, &d) == ACE_ERR_INVALID, "ppd");
  expect(ace_build(nullptr, &d, 1, &d, &d, &d) == ACE_ERR_INVALID, "build");
  expect(ace_build_targets(nullptr, &d, 1, &d, 1, &d, &d) == ACE_ERR_INVALID, "targets");
  expect(ace_apply(nullptr, &d, 1, &d, 1, &d) == ACE_ERR_INVALID, "apply");
  expect(ace_apply_noalloc(nullptr, &d, 1, &d, 1, &d) == ACE_ERR_INVALID, "apply_noalloc");
  expect(exchange_apply_direct(nullptr, &d, 1, &d, 1, &d) == ACE_ERR_INVALID, "direct");
  expect(tda_coupling(nullptr, &d, 1, &d, 1, 2, &d) == ACE_ERR_INVALID, "tda");
  expect(ace_trace_enable(nullptr, 1) == ACE_ERR_INVALID, "trace_enable");
  long long cnt = 0;
  expect(ace_trace_read(nullptr, 0, &d, &cnt) == ACE_ERR_INVALID, "trace_read");
  expect(ace_trace_reset(nullptr) == ACE_ERR_INVALID, "trace_reset");
  expect(scf_density(nullptr, &d, 1, &d) == ACE_ERR_INVALID, "density");
  expect(hartree_potential(nullptr, &d, &d) == ACE_ERR_INVALID, "hartree");
  double e5[5];
  expect(scf_energies(nullptr, &d, &d, 1, e5) == ACE_ERR_INVALID, "energies");
  ace_scf_opts so;
  std::memset(&so, 0, sizeof(so));
  ace_scf_result sr;
  expect(scf_run(nullptr, &d, &d, 1, &so, &sr, nullptr, nullptr) == ACE_ERR_INVALID, "scf_run");
  expect(strength_function(nullptr, nullptr, 1, 0.0, 0.1, 4, 0.1, nullptr, nullptr) ==
             ACE_ERR_INVALID,
         "strength");
  expect(sym_eig_small(0, nullptr, 1, nullptr, nullptr, 1, nullptr) == ACE_ERR_INVALID, "eig");

  // batches: argument checks, then a creation that needs a device
  ace_batch* b = nullptr;
  expect(ace_batch_create(7, nullptr, &b) == ACE_ERR_INVALID, "batch bad dtype");
  expect(ace_batch_create(0, nullptr, nullptr) == ACE_ERR_INVALID, "batch null out");
  expect(ace_batch_destroy(nullptr) == ACE_OK, "batch destroy null");
  expect(ace_build_batched(nullptr, nullptr, 1) == ACE_ERR_INVALID, "batched null");
  char buf[8];
  expect(ace_batch_tuning(nullptr, buf, (int)sizeof(buf)) == ACE_ERR_INVALID, "tuning null");
  int mol = 0;
  expect(ace_batch_status(nullptr, &st, &mol, &info) == ACE_ERR_INVALID, "batch status null");
  const int rb = ace_batch_create(1, nullptr, &b);
  if (rb == ACE_OK) {
    // host-side validation of the system list: bad edge, bad orbital count, null pointers
    std::vector<ace_mol> mols(3);
    for (auto& m : mols) {
      m.n = 16;
      m.h = 0.3;
      m.norb = 2;
      m.phi = &d;
      m.xi = &d;
      m.M = nullptr;
      m.ex = nullptr;
    }
    mols[1].n = 11;
    expect(ace_build_batched(b, mols.data(), 3) != ACE_OK, "batched bad edge");
    mols[1].n = 16;
    mols[2].norb = 0;
    expect(ace_build_batched(b, mols.data(), 3) == ACE_ERR_INVALID, "batched bad norb");
    mols[2].norb = 2;
    mols[0].phi = nullptr;
    expect(ace_build_batched(b, mols.data(), 3) == ACE_ERR_INVALID, "batched null phi");
    expect(ace_batch_tuning(b, buf, 1) == ACE_OK && buf[0] == 0, "tuning one byte");
    expect(ace_batch_destroy(b) == ACE_OK, "batch destroy");
  }

  // a context with valid arguments: on a machine without a device this is the failure path
  // (ACE_ERR_HIP or ACE_ERR_OOM after partial set-up); with a device, a real context
  const int rc = ace_ctx_create(16, 0.3, ACE_C64, nullptr, &ctx);
  expect(rc == ACE_OK || rc == ACE_ERR_HIP || rc == ACE_ERR_OOM, "create valid");
  if (rc == ACE_OK) {
    expect(ace_build(ctx, nullptr, 1, &d, nullptr, nullptr) == ACE_ERR_INVALID, "build null phi");
    expect(ace_build(ctx, &d, 33, &d, nullptr, nullptr) == ACE_ERR_INVALID, "build too many");
    const int32_t bad[2] = {0, 5};
    expect(pair_poisson_batched(ctx, &d, 1, &d, 1, bad, 1, &d) == ACE_ERR_INVALID, "pp range");
    expect(ace_ctx_destroy(ctx) == ACE_OK, "destroy");
  } else {
    expect(ctx == nullptr, "no context on failure");
  }
  ace_convnet* net = nullptr;
  expect(convnet_create(nullptr, nullptr) == ACE_ERR_INVALID, "convnet null out");
  const int rn = convnet_create(nullptr, &net);
  if (rn == ACE_OK) expect(convnet_destroy(net) == ACE_OK, "convnet destroy");

  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
