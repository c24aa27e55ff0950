// Host paths of the C ABI (argument validation, the policies of sections
// 4.1-4.2, status strings, server configuration) through a build of the
// library whose host code carries address and undefined-behaviour
// sanitizers.  Every call here returns before any HIP call: the device
// pointers are never dereferenced, and no GPU is needed.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/pf.h"

namespace {

int failures = 0;
#define CHECK(c)                                                                      \
  do {                                                                                \
    if (!(c)) {                                                                       \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c);      \
      ++failures;                                                                     \
    }                                                                                 \
  } while (0)

pf_desc good_desc() {
  pf_desc d;
  std::memset(&d, 0, sizeof(d));
  d.struct_size = sizeof(pf_desc);
  d.op = PF_OP_SYM;
  d.n = 256;
  d.p = 16;
  d.degree = 8;
  d.q = 1;
  d.a = -1.0;
  d.b = 0.5;
  d.work = PF_F32;
  return d;
}

pf_mat fake_mat(uintptr_t ptr = 0x10000, pf_dtype t = PF_F32, int64_t ld = 256) {
  pf_mat m;
  std::memset(&m, 0, sizeof(m));
  m.data = reinterpret_cast<const void*>(ptr);
  m.dtype = t;
  m.ld = ld;
  m.tile = 128;
  return m;
}

void* ptr(uintptr_t v) { return reinterpret_cast<void*>(v); }

void descriptors() {
  CHECK(pf_abi_version() == PF_ABI_VERSION);
  for (int s = 0; s <= 8; ++s) CHECK(std::strlen(pf_status_string((pf_status)s)) > 0);
  size_t bytes = 0;
  pf_desc d = good_desc();
  CHECK(pf_workspace_size(&d, &bytes) == PF_OK && bytes > 0);
  pf_desc bad = good_desc();
  bad.p = 0;
  CHECK(pf_workspace_size(&bad, &bytes) == PF_ERR_ARG && std::strlen(pf_last_error()) > 0);
  bad = good_desc();
  bad.a = bad.b;
  CHECK(pf_workspace_size(&bad, &bytes) == PF_ERR_ARG);
  bad = good_desc();
  bad.struct_size = 4;
  CHECK(pf_workspace_size(&bad, &bytes) == PF_ERR_ARG);
  bad = good_desc();
  bad.flags = 0x4000;
  CHECK(pf_workspace_size(&bad, &bytes) == PF_ERR_ARG);
  bad = good_desc();
  bad.flags = PF_FLAG_SCALED;             // needs spec_ub > b
  CHECK(pf_workspace_size(&bad, &bytes) == PF_ERR_ARG);
  CHECK(pf_workspace_size(nullptr, &bytes) == PF_ERR_ARG);
}

void extract_rejects() {
  pf_desc d = good_desc();
  pf_mat x = fake_mat(), r = fake_mat();
  CHECK(pf_extract(&d, nullptr, &r, ptr(0x20000), 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  pf_mat m = fake_mat();
  m.ld = 100;
  CHECK(pf_extract(&d, &m, &r, ptr(0x20000), 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  m = fake_mat(0x10004);
  CHECK(pf_extract(&d, &m, &r, ptr(0x20000), 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  m = fake_mat(0x10000, PF_F8E4M3);
  CHECK(pf_extract(&d, &m, &r, ptr(0x20000), 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  CHECK(pf_extract(&d, &x, &r, nullptr, 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) == PF_ERR_ARG);
  CHECK(pf_extract(&d, &x, &r, ptr(0x20000), 10, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  CHECK(pf_extract(&d, &x, &r, ptr(0x20000), 256, nullptr, nullptr, nullptr) == PF_ERR_ARG);
  CHECK(pf_extract_noalloc(&d, &x, &r, nullptr, 256, static_cast<double*>(ptr(0x30000)), nullptr, nullptr) ==
        PF_ERR_ARG);
  // a batch is validated as a whole before anything is enqueued
  pf_desc ds[2] = {good_desc(), good_desc()};
  ds[1].degree = 0;
  pf_mat xs[2] = {fake_mat(), fake_mat()};
  void* us[2] = {ptr(0x20000), ptr(0x28000)};
  int64_t ldus[2] = {256, 256};
  double* ths[2] = {static_cast<double*>(ptr(0x30000)), static_cast<double*>(ptr(0x38000))};
  CHECK(pf_extract_batch(2, ds, xs, xs, us, ldus, ths, nullptr, nullptr) == PF_ERR_ARG);
  CHECK(std::strstr(pf_last_error(), "block 1") != nullptr);
  CHECK(pf_extract_batch(-1, ds, xs, xs, us, ldus, ths, nullptr, nullptr) == PF_ERR_ARG);
}

void sessions_and_helpers() {
  CHECK(pf_session_close(nullptr) == PF_ERR_ARG);
  CHECK(pf_session_step(nullptr, nullptr, nullptr, nullptr, nullptr) == PF_ERR_ARG);
  CHECK(pf_session_set_interval(nullptr, -1.0, 1.0) == PF_ERR_ARG);
  CHECK(pf_session_set_filter(nullptr, 8, 1) == PF_ERR_ARG);
  pf_desc d = good_desc();
  pf_session* h = nullptr;
  CHECK(pf_session_open(&d, ptr(0x1000), 3, 0, &h) == PF_ERR_ARG);
  CHECK(pf_eigh(nullptr, 4, 4, static_cast<double*>(ptr(0x80000)), static_cast<double*>(ptr(0x100000)), 4,
                nullptr) == PF_ERR_ARG);
  CHECK(pf_eigh(static_cast<const double*>(ptr(0x10000)), 129, 129, static_cast<double*>(ptr(0x80000)),
                static_cast<double*>(ptr(0x100000)), 129, nullptr) == PF_ERR_ARG);
}

void server_config() {
  pf_server_config c;
  std::memset(&c, 0, sizeof(c));
  c.struct_size = sizeof(c);
  pf_server* s = nullptr;
  CHECK(pf_server_create(&c, &s) == PF_ERR_ARG);          // zero budget
  c.hbm_budget = size_t(1) << 30;
  c.streams = 65;
  CHECK(pf_server_create(&c, &s) == PF_ERR_ARG);
  c.streams = 0;
  c.max_batches = -1;
  CHECK(pf_server_create(&c, &s) == PF_ERR_ARG);
  c.max_batches = 0;
  c.reserved = 1;
  CHECK(pf_server_create(&c, &s) == PF_ERR_ARG);
  c.reserved = 0;
  c.flags = 0x80;
  CHECK(pf_server_create(&c, &s) == PF_ERR_ARG);
  CHECK(pf_server_destroy(nullptr) == PF_ERR_ARG);
  CHECK(pf_server_close(nullptr, 1) == PF_ERR_ARG);
}

void policies() {
  double a = 0, b = 0;
  CHECK(pf_interval_policy(-1.0, 0.0, 0.1, 0, 0.0, &a, &b) == PF_OK && a == -1.0 && b < 0.0);
  CHECK(pf_interval_policy(-1.0, 0.0, 1.5, 0, 0.0, &a, &b) == PF_ERR_ARG);
  int32_t p = 0;
  CHECK(pf_block_size_policy(10, 1.5, 0, 0, &p) == PF_OK && p == 20);
  CHECK(pf_block_size_policy(3, std::nan(""), 0, 0, &p) == PF_ERR_ARG);
  int32_t deg = 0;
  CHECK(pf_degree_policy(1.0, -5.0, 0.8, 1, 1e-6, 1, 64, &deg) == PF_OK && deg >= 1 && deg <= 64);
  CHECK(pf_degree_policy(0.5, -1.0, 0.8, 1, 1e-3, 1, 64, &deg) == PF_ERR_ARG);   // theta inside [a, b]
}

}  // namespace

int main() {
  descriptors();
  extract_rejects();
  sessions_and_helpers();
  server_config();
  policies();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("C-ABI host checks passed\n");
  return 0;
}
