// Exercises the library's host-only checks (mesh validation, checkpoint
// buffers) on valid and corrupted inputs; built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_checks.py.  Exits non-zero
// when a check gives an unexpected status; the sanitizers abort on any
// invalid memory access or undefined behaviour.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "tk_host.h"

namespace {

// An n x n x n box of unit cubes (h = 1/n), faces on the coordinate planes;
// the outer faces take boundary conditions 0..5 (one per side).
struct Box {
  std::vector<int> left, right;
  std::vector<double> normal, area, volume;
  std::vector<tk_bc> bc;
  tk_mesh_desc desc() {
    tk_mesh_desc d{};
    d.n_cells = (int32_t)volume.size();
    d.n_faces = (int32_t)left.size();
    d.face_left = left.data();
    d.face_right = right.data();
    d.face_normal = normal.data();
    d.face_area = area.data();
    d.cell_volume = volume.data();
    d.n_bc = (int32_t)bc.size();
    d.bc = bc.data();
    return d;
  }
};

Box make_box(int n, int side_kind) {
  Box b;
  const double h = 1.0 / n;
  auto id = [n](int i, int j, int k) { return i + n * (j + n * k); };
  for (int c = 0; c < n * n * n; ++c) b.volume.push_back(h * h * h);
  for (int s = 0; s < 6; ++s) {
    tk_bc bc{};
    bc.kind = side_kind;
    bc.n = 1.0;
    bc.T = 1.0;
    bc.T_w = 1.0;
    b.bc.push_back(bc);
  }
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i <= n; ++i) {
          // face i between cells i-1 and i along axis a
          int p[3];
          auto cell = [&](int ii) {
            p[a] = ii;
            p[(a + 1) % 3] = j;
            p[(a + 2) % 3] = k;
            return id(p[0], p[1], p[2]);
          };
          int L, R;
          if (i == 0) { L = cell(0); R = -(2 * a) - 1; }
          else if (i == n) { L = cell(n - 1); R = -(2 * a + 1) - 1; }
          else { L = cell(i - 1); R = cell(i); }
          double e[3] = {0, 0, 0};
          e[a] = (i == 0) ? -1.0 : 1.0;
          b.left.push_back(L);
          b.right.push_back(R);
          b.normal.insert(b.normal.end(), e, e + 3);
          b.area.push_back(h * h);
        }
  return b;
}

int failures = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "unexpected: %s\n", what);
    ++failures;
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(12345);
  std::string err;
  // valid meshes
  for (int kind : {TK_BC_SYM, TK_BC_INFLOW, TK_BC_OUTFLOW, TK_BC_WALL}) {
    Box b = make_box(3, kind);
    tk_mesh m;
    tk_mesh_desc d = b.desc();
    expect(tk::mesh_build_host(&d, &m, &err) == TK_OK, "valid box rejected");
  }
  // targeted corruptions with a known answer
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  {
    struct Case { const char* what; void (*mutate)(Box&); };
    static const Case cases[] = {
        {"NaN normal", [](Box& b) { b.normal[4] = std::numeric_limits<double>::quiet_NaN(); }},
        {"non-unit normal", [](Box& b) { b.normal[3] = 0.5; }},
        {"NaN area", [](Box& b) { b.area[7] = std::numeric_limits<double>::quiet_NaN(); }},
        {"infinite area", [](Box& b) { b.area[7] = std::numeric_limits<double>::infinity(); }},
        {"zero volume", [](Box& b) { b.volume[2] = 0.0; }},
        {"NaN volume", [](Box& b) { b.volume[2] = std::numeric_limits<double>::quiet_NaN(); }},
        {"face_left out of range", [](Box& b) { b.left[5] = (int)b.volume.size(); }},
        {"face_left negative", [](Box& b) { b.left[5] = -3; }},
        {"face_right INT_MIN", [](Box& b) { b.right[0] = INT_MIN; }},
        {"face_right out of range", [](Box& b) { b.right[40] = INT_MAX; }},
        {"face_right equals face_left", [](Box& b) {
           for (size_t j = 0; j < b.right.size(); ++j)
             if (b.right[j] >= 0) { b.right[j] = b.left[j]; break; }
         }},
        {"unknown bc kind", [](Box& b) { b.bc[1].kind = 17; }},
        {"open cell", [](Box& b) { b.area[0] *= 2.0; }},
        {"wall off the axes", [](Box& b) {
           for (auto& bc : b.bc) bc.kind = TK_BC_WALL;
           const double s = std::sqrt(0.5);
           b.normal[0] = -s; b.normal[1] = -s; b.normal[2] = 0.0;
         }},
    };
    for (const Case& c : cases) {
      Box b = make_box(3, TK_BC_OUTFLOW);
      c.mutate(b);
      tk_mesh m;
      tk_mesh_desc d = b.desc();
      if (tk::mesh_build_host(&d, &m, &err) != TK_EINVAL) {
        std::fprintf(stderr, "unexpected: %s accepted\n", c.what);
        ++failures;
      }
    }
    Box b = make_box(2, TK_BC_SYM);
    tk_mesh m;
    tk_mesh_desc d = b.desc();
    d.n_bc = -1;
    expect(tk::mesh_build_host(&d, &m, &err) == TK_EINVAL, "negative n_bc accepted");
    d = b.desc();
    d.face_normal = nullptr;
    expect(tk::mesh_build_host(&d, &m, &err) == TK_EINVAL, "missing normals accepted");
    expect(tk::mesh_build_host(nullptr, &m, &err) == TK_EINVAL, "null description accepted");
  }
  // random corruptions: any status, no invalid access
  int ok = 0, rejected = 0;
  for (int it = 0; it < 20000; ++it) {
    Box b = make_box(1 + (int)(rng() % 3), TK_BC_SYM + (int)(rng() % 4));
    const int edits = 1 + (int)(rng() % 4);
    for (int q = 0; q < edits; ++q) {
      const size_t nf = b.left.size(), nc = b.volume.size();
      const int vals[] = {INT_MIN, INT_MIN + 1, -7, -1, 0, 1, (int)nc - 1, (int)nc, INT_MAX};
      const double dv[] = {nan, inf, -inf, 0.0, -1.0, 1e-300, 1e300, 0.5, 1.0, -1.0};
      switch (rng() % 7) {
        case 0: b.left[rng() % nf] = vals[rng() % 9]; break;
        case 1: b.right[rng() % nf] = vals[rng() % 9]; break;
        case 2: b.normal[rng() % (3 * nf)] = dv[rng() % 10]; break;
        case 3: b.area[rng() % nf] = dv[rng() % 10]; break;
        case 4: b.volume[rng() % nc] = dv[rng() % 10]; break;
        case 5:
          if (!b.bc.empty()) b.bc[rng() % b.bc.size()].kind = (int32_t)(rng() % 9) - 2;
          break;
        case 6: b.bc.resize(rng() % 7); break;
      }
    }
    tk_mesh m;
    tk_mesh_desc d = b.desc();
    if (b.bc.empty()) d.bc = nullptr;
    (tk::mesh_build_host(&d, &m, &err) == TK_OK ? ok : rejected)++;
  }
  // checkpoint headers
  tk::CkptHeader want{};
  std::memcpy(want.magic, "TKCKPT2", 8);
  want.N = 16; want.CS = 6; want.nc = 10; want.ninst = 1;
  const size_t total = 4096;
  {
    std::vector<unsigned char> buf(total, 0);
    std::memcpy(buf.data(), &want, sizeof(want));
    expect(tk::ckpt_check_header(buf.data(), buf.size(), want, total, &err) == TK_OK, "valid header rejected");
    expect(tk::ckpt_check_header(buf.data(), total - 1, want, total, &err) == TK_EINVAL, "short buffer accepted");
    expect(tk::ckpt_check_header(buf.data(), 3, want, total, &err) == TK_EINVAL, "3-byte buffer accepted");
    expect(tk::ckpt_check_header(nullptr, total, want, total, &err) == TK_EINVAL, "null buffer accepted");
    buf[0] = 'X';
    expect(tk::ckpt_check_header(buf.data(), buf.size(), want, total, &err) == TK_EINVAL, "bad magic accepted");
  }
  for (int it = 0; it < 20000; ++it) {
    const size_t n = rng() % 96;
    std::vector<unsigned char> buf(n);
    for (auto& c : buf) c = (unsigned char)rng();
    if (n >= sizeof(want) && rng() % 2) {
      std::memcpy(buf.data(), &want, sizeof(want));
      buf[8 + rng() % (sizeof(want) - 8)] ^= (unsigned char)(1 + rng() % 255);
    }
    const tk_status s = tk::ckpt_check_header(buf.data(), n, want, total, &err);
    expect(s == TK_EINVAL, "random or corrupted header accepted");
  }
  // restored ranks
  for (int it = 0; it < 20000; ++it) {
    const int CS = 1 + (int)(rng() % 16);
    const size_t n = rng() % 40;
    std::vector<int> r(n);
    bool good = true;
    for (auto& v : r) {
      v = (rng() % 8 == 0) ? (int)(rng() % 40) - 10 : 1 + (int)(rng() % CS);
      good = good && v >= 1 && v <= CS;
    }
    const tk_status s = tk::ckpt_check_ranks(r.data(), n, CS, &err);
    expect((s == TK_OK) == good, "rank check disagrees");
  }
  std::printf("meshes: %d accepted, %d rejected; failures %d\n", ok, rejected, failures);
  return failures ? 1 : 0;
}
