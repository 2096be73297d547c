// Randomised check of the serving arena (paper_1101_0265_amd/csrc/arena.h) against a
// brute-force model that marks every 256-byte unit of the range as free or used.
// usage: arena_check SEED STEPS   -> prints "ok <allocs> <failed allocs>" or aborts.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1101_0265_amd/csrc/arena.h"

using snf::Arena;

static void fail(const char* what, long a, long b) {
  std::fprintf(stderr, "arena check failed: %s (%ld, %ld)\n", what, a, b);
  std::abort();
}

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  const int steps = argc > 2 ? std::atoi(argv[2]) : 20000;
  std::mt19937_64 rng(seed);
  const size_t U = Arena::kAlign;
  const size_t units = 64 + rng() % 4000;          // arena of `units` 256-byte units
  const size_t size = units * U;
  Arena a;
  a.init(size);
  std::vector<char> used(units, 0);                 // the model
  struct Live { size_t off, bytes; };
  std::vector<Live> live;
  long n_alloc = 0, n_fail = 0;
  auto model_first_fit = [&](size_t need) -> long {
    size_t run = 0;
    for (size_t u = 0; u < units; ++u) {
      run = used[u] ? 0 : run + 1;
      if (run == need) return (long)(u + 1 - need);
    }
    return -1;
  };
  for (int s = 0; s < steps; ++s) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      // sizes from 1 byte to a quarter of the arena, not multiples of 256 in general
      const size_t bytes = 1 + rng() % (size / 4);
      const size_t need = (bytes + U - 1) / U;
      const long expect = model_first_fit(need);
      size_t off = ~(size_t)0;
      const bool ok = a.alloc(bytes, &off);
      if (ok != (expect >= 0)) fail("alloc success differs from the model", (long)ok, expect);
      if (!ok) { ++n_fail; continue; }
      ++n_alloc;
      if (off % U) fail("offset not 256-byte aligned", (long)off, 0);
      if ((long)(off / U) != expect) fail("not the first fit", (long)(off / U), expect);
      if (off + need * U > size) fail("range past the end", (long)off, (long)need);
      for (size_t u = off / U; u < off / U + need; ++u) {
        if (used[u]) fail("overlaps a live range", (long)u, 0);
        used[u] = 1;
      }
      live.push_back({off, bytes});
    } else {
      const size_t k = rng() % live.size();
      const Live l = live[k];
      live[k] = live.back();
      live.pop_back();
      a.release(l.off, l.bytes);
      for (size_t u = l.off / U; u < l.off / U + (l.bytes + U - 1) / U; ++u) used[u] = 0;
    }
    // the free list is exactly the model's maximal free runs (coalesced, in order)
    if (s % 97 == 0 || s + 1 == steps) {
      auto it = a.free_ranges().begin();
      size_t u = 0;
      while (u < units) {
        if (used[u]) { ++u; continue; }
        size_t v = u;
        while (v < units && !used[v]) ++v;
        if (it == a.free_ranges().end()) fail("free run missing from the list", (long)u, (long)v);
        if (it->first != u * U || it->second != (v - u) * U)
          fail("free list differs from the model", (long)it->first, (long)(u * U));
        ++it;
        u = v;
      }
      if (it != a.free_ranges().end()) fail("extra free range", (long)it->first, 0);
    }
  }
  // releasing everything leaves one free range: the whole arena can be taken at once
  for (const Live& l : live) a.release(l.off, l.bytes);
  size_t off = 1;
  if (!a.alloc(size, &off) || off != 0) fail("arena not whole after releasing all", (long)off, 0);
  if (a.alloc(1, &off)) fail("alloc from a full arena", (long)off, 0);
  std::printf("ok %ld %ld\n", n_alloc, n_fail);
  return 0;
}
