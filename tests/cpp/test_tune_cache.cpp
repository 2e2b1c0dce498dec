// Host test of the autotuner's JSON-lines cache (tune_cache.h).
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../../paper_2606_21791_amd/csrc/tune_cache.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const char* path = argv[1];
  std::remove(path);
  // keys: primitive count bucket is ceil(log2 N)
  CHECK(sgtune::make_key("gfx950", 134826, 800, 800, 0, 3, 32, 512) == "gfx950|n18|800x800|f32|sh3|fb32|mb512");
  CHECK(sgtune::make_key("gfx950", 131072, 800, 800, 2, 0, 0, 256) == "gfx950|n17|800x800|bf16|sh0|fb0|mb256");
  CHECK(sgtune::make_key("gfx950", 1, 64, 48, 1, 1, 0, 0) == "gfx950|n0|64x48|f16|sh1|fb0|mb0");
  sgtune::Cfg c;
  double r = 0.0;
  CHECK(!sgtune::lookup(path, "k1", &c, &r));            // no file yet
  sgtune::Cfg a;
  a.tile = 8; a.batch = 128; a.streams = 32; a.threads = 4; a.wgs = 1; a.resume = 128; a.graphs = 1; a.grid = 64;
  CHECK(sgtune::append(path, "k1", a, 1234567.5));
  sgtune::Cfg b;
  b.tile = 32;
  CHECK(sgtune::append(path, "k2", b, 10.0));
  CHECK(sgtune::lookup(path, "k1", &c, &r));
  CHECK(c.tile == 8 && c.batch == 128 && c.streams == 32 && c.threads == 4 && c.wgs == 1 && c.resume == 128 &&
        c.graphs == 1 && c.grid == 64 && r > 1234567.0 && r < 1234568.0);
  CHECK(sgtune::lookup(path, "k2", &c, &r) && c.tile == 32 && c.batch == 32 && r == 10.0);
  CHECK(!sgtune::lookup(path, "k", &c, &r));             // keys match whole, not by prefix
  a.batch = 256;
  CHECK(sgtune::append(path, "k1", a, 5.0));            // a later entry overrides
  CHECK(sgtune::lookup(path, "k1", &c, &r) && c.batch == 256 && r == 5.0);
  std::FILE* f = std::fopen(path, "a");                  // a damaged line is skipped
  std::fputs("{\"key\": \"k2\", \"tile\": 8}\n", f);
  // a line without "grid" reads as grid 0
  std::fputs("{\"key\": \"k3\", \"tile\": 16, \"batch\": 64, \"streams\": 8, \"threads\": 2, "
             "\"wgs_per_cu\": 2, \"resume\": 64, \"graphs\": 0, \"inj_per_s\": 7}\n", f);
  std::fclose(f);
  CHECK(sgtune::lookup(path, "k2", &c, &r) && c.tile == 32);
  CHECK(sgtune::lookup(path, "k3", &c, &r) && c.batch == 64 && c.grid == 0 && r == 7.0);
  std::printf("tune cache ok\n");
  return 0;
}
