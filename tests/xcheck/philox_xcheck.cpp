// Independent Philox4x32-10 evaluator for the oracle's cross-check.
// Built twice: with -DUSE_TORCH against PyTorch's ATen philox_engine header,
// and with -DUSE_ROCRAND against rocRAND's philox4x32_10_engine header.
// Reads n records of (ctr[4], key[2]) uint32 from argv[1] and writes n
// records of out[4] uint32 to argv[2]. Counter word mapping for both:
// (offset lo, offset hi, subsequence lo, subsequence hi), key = seed.
#include <cstdint>
#include <cstdio>
#include <vector>
#if defined(USE_TORCH)
#include <ATen/core/PhiloxRNGEngine.h>
#elif defined(USE_ROCRAND)
#include <rocrand/rocrand_philox4x32_10.h>
#else
#error "define USE_TORCH or USE_ROCRAND"
#endif

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  std::vector<uint32_t> in;
  uint32_t rec[6];
  while (std::fread(rec, sizeof(uint32_t), 6, f) == 6) in.insert(in.end(), rec, rec + 6);
  std::fclose(f);
  const size_t n = in.size() / 6;
  std::vector<uint32_t> out(4 * n);
  for (size_t j = 0; j < n; ++j) {
    const uint32_t* r = &in[6 * j];
    const uint64_t offset = uint64_t(r[0]) | (uint64_t(r[1]) << 32);
    const uint64_t subseq = uint64_t(r[2]) | (uint64_t(r[3]) << 32);
    const uint64_t seed = uint64_t(r[4]) | (uint64_t(r[5]) << 32);
#if defined(USE_TORCH)
    at::philox_engine e(seed, subseq, offset);
    for (int w = 0; w < 4; ++w) out[4 * j + w] = e();
#else
    // rocRAND counts its offset in 32-bit outputs, four per block.
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset * 4ull);
    const uint4 b = e.next4();
    out[4 * j + 0] = b.x; out[4 * j + 1] = b.y; out[4 * j + 2] = b.z; out[4 * j + 3] = b.w;
#endif
  }
  FILE* g = std::fopen(argv[2], "wb");
  if (!g) return 4;
  std::fwrite(out.data(), sizeof(uint32_t), out.size(), g);
  std::fclose(g);
  return 0;
}
