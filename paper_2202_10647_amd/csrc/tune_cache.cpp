// Autotuner cache file of the batched plan (see tune_cache.hpp).
#include "tune_cache.hpp"

#include <cstdio>
#include <cstring>

namespace adk {

int tune_cache_lookup(const char *path, const std::string &key)
{
    if (!path) return 0;
    FILE *f = std::fopen(path, "r");
    if (!f) return 0;
    // The last valid entry of a key wins.  A line that does not parse (a
    // truncated write, another program's file, a value other than 1, 2 or 4)
    // is skipped and the lines after it are still read, so a key with no
    // valid entry is tuned again and the others keep their choice.
    char line[1024], k[512], extra = 0;
    int v = 0, found = 0;
    while (std::fgets(line, sizeof(line), f)) {
        const size_t len = std::strlen(line);
        if (len + 1 == sizeof(line) && line[len - 1] != '\n') {  // longer than any entry: drop the rest
            int c;
            while ((c = std::fgetc(f)) != EOF && c != '\n') {
            }
            continue;
        }
        if (std::sscanf(line, "%511s %d %c", k, &v, &extra) == 2 && key == k && (v == 1 || v == 2 || v == 4))
            found = v;
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const char *path, const std::string &key, int cpl)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), cpl);
    std::fclose(f);
}

}  // namespace adk
