"""Host-side logic that needs no GPU: serving admission and footprints, and
kernel-header helpers compiled for the host."""
import pytest

from paper_1812_01502_amd.serving import CTL_BYTES, PARAM_BYTES, StreamRequest, plan_admission, slot_footprint


def test_control_and_parameter_sizes_match_the_device_structs():
    """The footprint constants equal sizeof(Ctl) and sizeof(ModelParams<float>)."""
    import os
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = (
        "#define __device__\n#define __host__\n#define __forceinline__ inline\n"
        "#include <cstdint>\n#include <cstdio>\n"
        f'#include "{root}/include/pf.h"\n'
        "namespace pfk { constexpr int kMaxDim = PF_MAX_DIM; }\n"
    )
    # the two structs are plain data: compile their definitions out of pf_device.h
    dev = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_device.h")).read()
    import re
    mp = re.search(r"template <typename T> struct ModelParams \{.*?\n\};", dev, re.S).group(0)
    consts = "\n".join(re.findall(r"constexpr int k(?:Off\w+|MaxPending) = [^;]+;", dev))
    ctl = re.search(r"struct Ctl \{.*?\n\};", dev, re.S).group(0)
    src += "namespace pfk {\n" + consts + "\n" + mp + "\n" + ctl + "\n}\n"
    src += 'int main(){printf("%zu %zu\\n", sizeof(pfk::Ctl), sizeof(pfk::ModelParams<float>));}\n'
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-std=c++17", os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    assert (int(out[0]), int(out[1])) == (CTL_BYTES, PARAM_BYTES)


def test_slot_footprint_counts_every_buffer():
    # states (2 buffers x d planes) + log-weights (2 buffers) + partial records,
    # each rounded to 64 floats as the library allocates them, + control block
    # + model parameters + record
    assert slot_footprint(1, 4096) == 4 * (2 * 4096 + 2 * 4096 + 64) + CTL_BYTES + PARAM_BYTES + 304
    assert slot_footprint(16, 1 << 20) > slot_footprint(4, 1 << 20) > slot_footprint(1, 1 << 20)


def _req(i, model, n):
    return StreamRequest(stream_id=i, model=model, n_particles=n, observations=None)


def _plan(waiting, shapes, nbytes, budget, fps, free=None):
    s_shape = list(shapes)
    s_bytes = list(nbytes)
    free = list(range(len(shapes))) if free is None else free
    out = plan_admission(waiting, free, s_shape, s_bytes, budget,
                         lambda r: fps.get((r.model, r.n_particles)))
    return out, s_shape, s_bytes


def test_admission_by_footprint_any_shape():
    """Streams of any shape are admitted while their footprints fit the
    budget; the rest wait; one larger than the budget is rejected."""
    fps = {("sv", 4096): 100, ("lg4", 1 << 20): 700, ("lg16", 1 << 16): 250, ("sv", 1 << 24): 5000}
    w = [_req(0, "sv", 4096), _req(1, "lg4", 1 << 20), _req(2, "lg16", 1 << 16), _req(3, "sv", 1 << 24),
         _req(4, "sv", 4096), _req(5, "nope", 4096)]
    (bind, rel, still, rej), shape, nb = _plan(w, [None] * 4, [0] * 4, 1000, fps)
    assert [r.stream_id for _, r in bind] == [0, 1, 4]      # 100 + 700 + 100 <= 1000; 250 waits
    assert [r.stream_id for r in still] == [2]
    assert sorted(r.stream_id for r, _ in rej) == [3, 5]
    assert sum(nb) == 900 and rel == []
    assert all(shape[s] == (r.model, r.n_particles) for s, r in bind)


def test_admission_reuses_and_releases_free_slots():
    """A free slot already holding the stream's shape is reused without new
    memory; otherwise the memory of free slots is given back (largest first)
    until the new stream fits; active slots are never touched."""
    fps = {("sv", 4096): 100, ("lg4", 1 << 20): 700}
    shapes = [("sv", 4096), ("lg4", 1 << 20), ("sv", 4096), None]
    nbytes = [100, 700, 100, 0]
    # slot 2 is active (not free); the budget is full but for 100 bytes
    (bind, rel, still, rej), shape, nb = _plan([_req(0, "sv", 4096)], shapes, nbytes, 1000, fps, free=[0, 1, 3])
    assert bind[0][0] == 0 and rel == [] and nb == [100, 700, 100, 0]
    (bind, rel, still, rej), shape, nb = _plan([_req(1, "lg4", 1 << 20), _req(2, "lg4", 1 << 20)],
                                              shapes, nbytes, 1000, fps, free=[0, 3])
    # slot 1 is busy: the first lg4 stream needs 700 with 100 left -> slot 0's
    # 100 bytes are not enough, so it waits; so does the second
    assert bind == [] and [r.stream_id for r in still] == [1, 2]
    (bind, rel, still, rej), shape, nb = _plan([_req(1, "lg4", 1 << 20)], shapes, nbytes, 1500, fps,
                                              free=[0, 3])
    assert bind[0][0] == 3 and rel == [0] and nb == [0, 700, 100, 700] and shape[0] is None
    assert sum(nb) <= 1500


def test_tile_coordinates_cover_every_particle_once():
    """The step kernel's tile geometry (tile_geo, pair_coords), compiled for
    the host from the kernel header: for every radix, stride and tile size
    the planner can choose (including one group per tile at stride 1), each
    particle pair's rows and columns lie inside the tile, map back to the
    pair's global indices, and the tiles of a stage cover every particle
    exactly once."""
    import os
    import re
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ker = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_kernels.h")).read()
    geo = re.search(r"struct TileGeo \{.*?\n\};\n.*?\n}\n.*?pair_coords\(.*?\n}\n", ker, re.S).group(0)
    src = ("#define __device__\n#define __host__\n#define __forceinline__ inline\n"
           "#include <cstdint>\n#include <cstdio>\n#include <vector>\n" + geo + r'''
int main() {
  long bad = 0, cases = 0;
  for (uint32_t log2N : {11u, 12u, 13u, 15u})
  for (uint32_t log2r = 1; log2r <= 12 && log2r < log2N; ++log2r)
  for (uint32_t log2R = 0; log2R + log2r <= log2N; log2R += (log2R ? log2R : 1))
  for (uint32_t log2E : {log2r, log2r + 1, 7u, 9u, 10u, 11u, 12u, 13u}) {
    if (log2E < log2r || log2E > log2N) continue;
    if (log2E == log2r && log2R != 0) continue;  // one group per tile only at stride 1
    const uint32_t log2C = log2E - log2r, C = 1u << log2C, r = 1u << log2r, E = 1u << log2E;
    std::vector<int> seen(1u << log2N, 0);
    for (uint32_t t = 0; t < (1u << (log2N - log2E)); ++t) {
      const TileGeo g = tile_geo(t, log2r, log2R, log2C);
      for (uint32_t f = 0; f < E; f += 2) {
        uint32_t q0, c0, q1, c1;
        uint64_t gi;
        pair_coords(g, f, q0, c0, q1, c1, gi);
        ++cases;
        if (q0 >= r || q1 >= r || c0 >= C || c1 >= C || gi + 1 >= (1ull << log2N)) { ++bad; continue; }
        auto back = [&](uint32_t q, uint32_t c) {
          return g.base + ((uint64_t)q << log2R) +
                 (g.wide ? c : ((uint64_t)(c >> log2R) << (log2r + log2R)) + (c & ((1u << log2R) - 1u)));
        };
        if (back(q0, c0) != gi || back(q1, c1) != gi + 1) ++bad;
        seen[gi]++;
        seen[gi + 1]++;
      }
    }
    for (int v : seen) if (v != 1) { ++bad; break; }
  }
  printf("%ld %ld\n", cases, bad);
  return 0;
}
''')
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "g.cpp"), "w").write(src)
        subprocess.run([cxx, "-O2", "-std=c++17", os.path.join(d, "g.cpp"), "-o", os.path.join(d, "g")], check=True)
        out = subprocess.run([os.path.join(d, "g")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    cases, bad = int(out[0]), int(out[1])
    assert cases > 1_000_000 and bad == 0, (cases, bad)


def test_padded_search_of_the_wide_group_path():
    """The draw of the r > 64 tile path (padded_search), compiled for the host
    from the kernel header: on a column whose member q sits at word
    q + q / 64, it returns what a plain binary search over the unpadded
    cumulative weights returns (the number of members <= target, at most
    r - 1), for every radix 128 .. 4096, with ties, zero weights, targets
    at and beyond the ends."""
    import os
    import re
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ker = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_kernels.h")).read()
    fn = re.search(r"template <int LR, typename T>\n__device__ __forceinline__ uint32_t padded_search\(.*?\n}\n",
                   ker, re.S).group(0)
    src = ("#define __device__\n#define __forceinline__ inline\n"
           "#include <cstdint>\n#include <cstdio>\n#include <random>\n#include <vector>\n" + fn + r'''
template <int LR> long check(std::mt19937& g, long& cases) {
  const uint32_t r = 1u << LR;
  long bad = 0;
  std::vector<float> cdf(r), col(r + r / 64);
  for (int trial = 0; trial < 200; ++trial) {
    float acc = 0.f;
    for (uint32_t q = 0; q < r; ++q) {
      const uint32_t kind = g() % 8u;
      acc += kind == 0 ? 0.f : (kind == 1 ? 1.f : (float)(g() % 1000u) * 1e-3f);
      cdf[q] = acc;
      col[q + q / 64] = acc;
    }
    for (int k = 0; k < 256; ++k) {
      float t;
      const uint32_t sel = g() % 4u;
      if (sel == 0) t = cdf[g() % r];                   // exactly a cumulative weight
      else if (sel == 1) t = acc * (float)(g() % 1000001u) * 1e-6f;
      else if (sel == 2) t = -1.f;
      else t = acc * 2.f + 1.f;
      uint32_t pos = 0;
      for (uint32_t s = r >> 1; s >= 1u; s >>= 1)
        if (cdf[pos + s - 1u] <= t) pos += s;
      ++cases;
      if (padded_search<LR>(col.data(), t) != pos) ++bad;
    }
  }
  return bad;
}
int main() {
  std::mt19937 g(7);
  long cases = 0, bad = 0;
  bad += check<7>(g, cases); bad += check<8>(g, cases); bad += check<9>(g, cases);
  bad += check<10>(g, cases); bad += check<11>(g, cases); bad += check<12>(g, cases);
  printf("%ld %ld\n", cases, bad);
  return 0;
}
''')
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-O2", "-std=c++17", os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    cases, bad = int(out[0]), int(out[1])
    assert cases == 6 * 200 * 256 and bad == 0


def test_global_draw_tile_positions():
    """The position search of the global path's draw (tile_positions), built
    for the host from the kernel header with AddressSanitizer: on tiles whose
    coarse levels hold every 16th and every 256th entry of the tile CDF in the
    device layout (global_cc_offset), it returns what a plain binary search
    of the tile CDF returns (the number of entries <= target, at most E - 1)
    for every tile size the runtime uses (E = 128 .. 4096), with the CDF
    contiguous or in runs of 16 paired with 16 other values, with zero weights,
    ties, targets equal to an entry, below the first and above the last; no
    read leaves the arrays as the runtime sizes them."""
    import os
    import re
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ker = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_kernels.h")).read()
    parts = [re.search(r"__host__ __device__ constexpr uint64_t global_cc_offset\(.*?\n", ker).group(0),
             re.search(r"__host__ __device__ constexpr uint64_t global_coarse_elems\(.*?\n}\n", ker, re.S).group(0),
             re.search(r"template <typename T, int ALIGN>\n__device__ __forceinline__ uint32_t count_le16\(.*?\n}\n",
                       ker, re.S).group(0),
             re.search(r"template <typename T, int NP, bool PAIRED>\n__device__ __forceinline__ void tile_positions\("
                       r".*?\n}\n", ker, re.S).group(0)]
    src = ("#define __device__\n#define __host__\n#define __forceinline__ inline\n"
           "#include <cstdint>\n#include <cstddef>\n#include <cstdio>\n#include <random>\n#include <vector>\n"
           "#include <cmath>\n" + "\n".join(parts) + r'''
template <bool PAIRED>
long check(uint32_t lg_e, uint32_t nt, std::mt19937& g, long& cases) {
  const uint32_t E = 1u << lg_e;
  const uint64_t N = (uint64_t)E * nt;
  long bad = 0;
  for (int trial = 0; trial < 40; ++trial) {
    std::vector<float> cdf(N), coarse(global_coarse_elems(N, nt)), dev(PAIRED ? 2 * N : N);
    float* cc = coarse.data() + global_cc_offset(N);
    for (uint32_t b = 0; b < nt; ++b) {
      float acc = 0.f;
      for (uint32_t q = 0; q < E; ++q) {
        const uint32_t kind = g() % 8u;
        acc += kind < 2 ? 0.f : (kind == 2 ? 1.f : (float)(g() % 1000u) * 1e-3f);
        const uint64_t i = (uint64_t)b * E + q;
        cdf[i] = acc;
        dev[PAIRED ? 2 * (i & ~(uint64_t)15) + (i & 15) : i] = acc;
        if (PAIRED) dev[2 * (i & ~(uint64_t)15) + 16 + (i & 15)] = -7.f;   // the paired states
        if ((q & 15u) == 15u) coarse[i >> 4] = acc;
        if ((q & 255u) == 255u) cc[(size_t)b * 16u + (q >> 8)] = acc;
      }
    }
    for (int k = 0; k < 64; ++k) {
      constexpr int NP = 4;
      uint32_t bb[NP];
      float lt[NP];
      uint64_t want[NP], got[NP];
      for (int e = 0; e < NP; ++e) {
        bb[e] = g() % nt;
        const float* t = cdf.data() + (uint64_t)bb[e] * E;
        const uint32_t sel = g() % 5u;
        lt[e] = sel == 0 ? t[g() % E] : sel == 1 ? t[E - 1] * (float)(g() % 1000001u) * 1e-6f
              : sel == 2 ? -1.f : sel == 3 ? t[E - 1] + 1.f : INFINITY;
        uint32_t pos = 0;
        for (uint32_t s = E >> 1; s >= 1u; s >>= 1)
          if (t[pos + s - 1u] <= lt[e]) pos += s;
        want[e] = (uint64_t)bb[e] * E + pos;
      }
      tile_positions<float, NP, PAIRED>(cc, coarse.data(), dev.data(), bb, lt, lg_e, got);
      for (int e = 0; e < NP; ++e) {
        ++cases;
        if (got[e] != want[e]) ++bad;
      }
    }
  }
  return bad;
}
int main() {
  std::mt19937 g(11);
  long cases = 0, bad = 0;
  for (uint32_t lg_e : {7u, 9u, 10u, 11u, 12u})
    for (uint32_t nt : {1u, 3u}) bad += check<false>(lg_e, nt, g, cases) + check<true>(lg_e, nt, g, cases);
  printf("%ld %ld\n", cases, bad);
  return 0;
}
''')
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    cases, bad = int(out[0]), int(out[1])
    assert cases == 2 * 5 * 2 * 40 * 64 * 4 and bad == 0, (cases, bad)


def test_systematic_global_plan_and_offspring_ranges():
    """The systematic global draw's plan and offspring ranges, built for the
    host from the kernel header with AddressSanitizer: the first output of
    every weight tile (sys_first_output, made non-decreasing), the items of
    at most kSysItem outputs that the prefix kernel writes, and per item the
    count of outputs below each CDF value (sys_outputs_below), whose
    differences give each particle its outputs: every output is written
    exactly once and gets exactly the ancestor of a plain search (the tile is
    the number of tile prefixes <= the target, the position the number of the
    tile's CDF entries <= the target's in-tile value, at most E - 1; a target
    at the total takes the last particle). Tile sizes 128 .. 4096, zero-weight
    tiles and particles, ties, weight concentrated on one tile (items split)
    and on the last particle; no read or write leaves the arrays."""
    import os
    import re
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ker = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_kernels.h")).read()
    parts = [re.search(r"constexpr uint32_t kSysItem = .*?\n", ker).group(0),
             re.search(r"__host__ __device__ constexpr uint64_t sys_max_items\(.*?\n}\n", ker, re.S).group(0),
             re.search(r"__device__ __forceinline__ double sys_target\(.*?\n}\n", ker, re.S).group(0),
             re.search(r"__device__ inline uint64_t sys_first_output\(.*?\n}\n", ker, re.S).group(0),
             re.search(r"template <typename T>\n__device__ __forceinline__ T sys_value\(.*?\n}\n", ker, re.S).group(0),
             re.search(r"template <typename T>\n__device__ inline uint32_t sys_outputs_below\(.*?\n}\n",
                       ker, re.S).group(0)]
    src = ("#define __device__\n#define __host__\n#define __forceinline__ inline\n"
           "#include <cstdint>\n#include <cstddef>\n#include <cstdio>\n#include <random>\n#include <vector>\n"
           "#include <cmath>\n#include <algorithm>\n" + "\n".join(parts) + r'''
// mode 0: mixed weights; 1: one tile holds almost all; 2: the last particle holds almost all
long check(uint32_t E, uint32_t nt, int mode, std::mt19937& g, long& cases) {
  const uint64_t N = (uint64_t)E * nt;
  std::vector<float> cdf(N);
  std::vector<double> pre(nt + 1), rs(nt);
  pre[0] = 0.0;
  const uint32_t heavy = g() % nt;
  for (uint32_t b = 0; b < nt; ++b) {
    float acc = 0.f;
    for (uint32_t q = 0; q < E; ++q) {
      const uint32_t kind = g() % 8u;
      float w = kind < 2 ? 0.f : (kind == 2 ? 1.f : (float)(g() % 1000u) * 1e-3f);
      if (mode == 2) w = (b == nt - 1 && q == E - 1) ? 1.f : 1e-9f;
      acc += w;
      cdf[(uint64_t)b * E + q] = acc;
    }
    double ev = (g() % 6u == 0u) ? 0.0 : std::ldexp(1.0 + (double)(g() % 1000u) * 1e-3, -(int)(g() % 8u));
    if (mode == 1) ev = b == heavy ? 1.0 : 1e-7;
    if (mode == 2) ev = 1.0;
    rs[b] = 1.0 / ev;
    pre[b + 1] = pre[b] + ev * (double)acc;
  }
  const double total = pre[nt];
  if (!(total > 0.0)) return 0;
  const double scale = total / (double)N, inv_scale = (double)N / total;
  long bad = 0;
  for (int trial = 0; trial < 6; ++trial) {
    const double u0 = (double)(g() >> 8) * 0x1p-24;
    // plan: first output per tile, non-decreasing; then the items
    std::vector<uint32_t> first(nt + 1);
    uint32_t omax = 0;
    for (uint32_t b = 0; b < nt; ++b) {
      const uint32_t o = (uint32_t)sys_first_output(pre[b], u0, scale, inv_scale, N);
      omax = std::max(omax, o);
      first[b] = omax;
    }
    first[nt] = (uint32_t)N;
    std::vector<uint32_t> items;
    for (uint32_t b = 0; b < nt; ++b)
      for (uint32_t o = first[b]; o < first[b + 1]; o += kSysItem) { items.push_back(b); items.push_back(o); }
    if (items.size() / 2 > sys_max_items(N, nt)) ++bad;
    std::vector<int64_t> anc(N, -1);
    for (size_t w = 0; w < items.size() / 2; ++w) {
      const uint32_t b = items[2 * w], start = items[2 * w + 1];
      const uint32_t lim = first[b + 1];
      const uint32_t end = lim - start > kSysItem ? start + kSysItem : lim;
      const uint32_t n = end - start;
      const float* t = cdf.data() + (uint64_t)b * E;
      std::vector<uint16_t> sf(E);
      std::vector<int> spos(n, -1);
      for (uint32_t q = 0; q < E; ++q)
        sf[q] = (uint16_t)sys_outputs_below<float>(t[q], n, start, u0, u0 + (double)start, scale, inv_scale,
                                                   total, pre[b], rs[b], 1.0 / rs[b]);
      for (uint32_t q = 0; q < E; ++q) {
        const uint32_t lo = q == 0 ? 0u : sf[q - 1], hi = q == E - 1 ? n : sf[q];
        for (uint32_t j = lo; j < hi; ++j) {
          if (spos.at(j) != -1) ++bad;   // an output written twice
          spos.at(j) = (int)q;
        }
      }
      for (uint32_t j = 0; j < n; ++j) {
        if (spos[j] < 0) { ++bad; continue; }   // an output never written
        if (anc[start + j] != -1) ++bad;
        anc[start + j] = (int64_t)b * E + spos[j];
      }
    }
    // the plain search
    for (uint64_t i = 0; i < N; ++i) {
      ++cases;
      const double tg = sys_target(i, u0, scale);
      uint32_t b = 0;
      for (uint32_t k = 1; k <= nt; ++k) if (pre[k] <= tg) b = k;
      float lt;
      if (b >= nt) { b = nt - 1; lt = INFINITY; } else { lt = (float)((tg - pre[b]) * rs[b]); }
      uint32_t c = 0;
      for (uint32_t q = 0; q < E; ++q) c += cdf[(uint64_t)b * E + q] <= lt ? 1u : 0u;
      const int64_t want = (int64_t)b * E + std::min(c, E - 1u);
      if (anc[i] != want) ++bad;
    }
  }
  return bad;
}
int main() {
  std::mt19937 g(5);
  long cases = 0, bad = 0;
  for (uint32_t E : {128u, 512u, 1024u, 2048u, 4096u})
    for (uint32_t nt : {1u, 4u, 9u})
      for (int mode : {0, 1, 2}) bad += check(E, nt, mode, g, cases);
  bad += check(128u, 160u, 1, g, cases) + check(4096u, 5u, 1, g, cases);
  printf("%ld %ld\n", cases, bad);
  return 0;
}
''')
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    cases, bad = int(out[0]), int(out[1])
    assert cases > 1_000_000 and bad == 0, (cases, bad)


def test_xcd_tile_order_is_a_permutation():
    """The XCD-aware block order (xcd_tile), built for the host from the
    kernel header: for every grid size up to 4100 it is a permutation of the
    blocks, and when the size is a multiple of 8 each XCD (block b on XCD
    b mod 8) gets one contiguous range of tiles."""
    import os
    import re
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ker = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_kernels.h")).read()
    fn = re.search(r"__device__ __forceinline__ uint32_t xcd_tile\(.*?\n}\n", ker, re.S).group(0)
    src = ("#define __device__\n#define __forceinline__ inline\n#include <cstdint>\n#include <cstdio>\n"
           "#include <vector>\n" + fn + r'''
int main() {
  long bad = 0;
  for (uint32_t n = 1; n <= 4100; ++n) {
    std::vector<int> seen(n, 0);
    for (uint32_t b = 0; b < n; ++b) {
      const uint32_t t = xcd_tile(b, n);
      if (t >= n || seen[t]++) ++bad;
    }
    if (n % 8 == 0)
      for (uint32_t x = 0; x < 8; ++x)
        for (uint32_t j = 1; j < n / 8; ++j)
          if (xcd_tile(x + 8 * j, n) != xcd_tile(x + 8 * (j - 1), n) + 1) ++bad;
  }
  printf("%ld\n", bad);
  return 0;
}
''')
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    assert int(out[0]) == 0
