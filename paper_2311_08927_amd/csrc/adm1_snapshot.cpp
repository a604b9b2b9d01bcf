// Binary particle snapshots: the per-interval exchange of particle data with
// the flow solver (sec. 2.3: positions, velocities and densities of the SPH
// particles are loaded every coupling step).  The paper reads and writes
// ASCII files and names that I/O as one of the main bottlenecks, about 4 s to
// read and 7.5 s to write per million particles (sec. 4.3), with binary files
// as the planned fix.  The layout (little endian) is:
//   64-byte header: "ADM1SNAP", uint32 version (1), uint32 field mask,
//                   uint64 n, float64 time (s), 32 zero bytes;
//   then, for each field present in mask-bit order, its rows of n values:
//   positions float32 [3][n] (m), velocities float32 [3][n] (m/s),
//   densities float32 [n] (kg/m3), ADM1 states float64 [35][n].
// Rows are moved with positional reads and writes in chunks of kChunk bytes
// spread over up to kThreads threads, straight between the file and the
// caller's (ideally pinned) host buffers.
#include <fcntl.h>
#include <stdint.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstring>
#include <thread>
#include <vector>

#include "adm1.h"

namespace {

constexpr char kMagic[8] = {'A', 'D', 'M', '1', 'S', 'N', 'A', 'P'};
constexpr uint32_t kVersion = 1;
constexpr int64_t kHeader = 64;
constexpr int64_t kChunk = 8 << 20;
constexpr int kThreads = 8;

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t fields;
    uint64_t n;
    double time_s;
    uint8_t reserved[32];
};
static_assert(sizeof(Header) == kHeader, "snapshot header is 64 bytes");

// One contiguous piece of the file and the host memory it maps to.
struct Piece {
    int64_t off;
    char* buf;
    int64_t bytes;
};

struct Field {
    uint32_t bit;
    int rows;
    int64_t elem;
};

constexpr Field kFields[4] = {{ADM1_SNAP_POS, 3, 4}, {ADM1_SNAP_VEL, 3, 4},
                              {ADM1_SNAP_RHO, 1, 4}, {ADM1_SNAP_STATE, 35, 8}};

// Move every piece with pread/pwrite in chunks, on up to kThreads threads.
// False on an I/O error; thread or memory exhaustion also ends in false
// (nothing is thrown across the C interface).
bool transfer(int fd, const std::vector<Piece>& pieces, bool write) noexcept
try {
    std::vector<Piece> chunks;
    for (const Piece& p : pieces)
        for (int64_t o = 0; o < p.bytes; o += kChunk)
            chunks.push_back({p.off + o, p.buf + o, std::min(kChunk, p.bytes - o)});
    std::atomic<size_t> next{0};
    std::atomic<bool> ok{true};
    auto work = [&]() {
        for (size_t k = next++; k < chunks.size() && ok; k = next++) {
            const Piece& c = chunks[k];
            int64_t done = 0;
            while (done < c.bytes) {
                const ssize_t r = write ? pwrite(fd, c.buf + done, c.bytes - done, c.off + done)
                                        : pread(fd, c.buf + done, c.bytes - done, c.off + done);
                if (r < 0 && errno == EINTR) continue;
                if (r <= 0) {
                    ok = false;
                    return;
                }
                done += r;
            }
        }
    };
    const int nt = (int)std::min<size_t>(kThreads, std::max<size_t>(1, chunks.size()));
    std::vector<std::thread> pool;
    pool.reserve(nt);
    try {
        for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    } catch (...) {
        // fewer helper threads than asked for: the ones started and this
        // thread still finish every chunk
    }
    work();
    for (auto& t : pool) t.join();
    return ok;
} catch (...) {
    return false;
}

int read_header(int fd, Header& h)
{
    if (pread(fd, &h, sizeof(h), 0) != (ssize_t)sizeof(h)) return ADM1_E_IO;
    if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion ||
        (h.fields & ~15u) != 0 || h.n > (uint64_t)INT64_MAX / 512)
        return ADM1_E_IO;
    return ADM1_OK;
}

// The fields of a checked header whose destinations are non-NULL.
int read_fields(int fd, const Header& h, int64_t ld, void* const dst[4]) noexcept
try {
    const int64_t n = (int64_t)h.n;
    std::vector<Piece> pieces;
    int64_t off = kHeader;
    int rc = ADM1_OK;
    for (int f = 0; f < 4; ++f) {
        const bool present = (h.fields & kFields[f].bit) != 0;
        if (dst[f] && !present) rc = ADM1_E_IO;
        if (!present) continue;
        for (int r = 0; r < kFields[f].rows; ++r) {
            if (dst[f])
                pieces.push_back({off, (char*)dst[f] + (int64_t)r * ld * kFields[f].elem,
                                  n * kFields[f].elem});
            off += n * kFields[f].elem;
        }
    }
    struct stat st;
    if (!rc && ld < n) rc = ADM1_E_SIZE;
    if (!rc && (fstat(fd, &st) != 0 || st.st_size != off)) rc = ADM1_E_IO;
    if (!rc && !transfer(fd, pieces, false)) rc = ADM1_E_IO;
    return rc;
} catch (...) {
    return ADM1_E_IO;
}

}  // namespace

extern "C" {

int adm1_snapshot_write(const char* path, int64_t n, int64_t ld, double time_s, const float* pos,
                        const float* vel, const float* rho, const double* state)
try {
    if (!path) return ADM1_E_NULL;
    if (n < 0 || ld < n || ld < 1) return ADM1_E_SIZE;
    Header h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.n = (uint64_t)n;
    h.time_s = time_s;
    const void* src[4] = {pos, vel, rho, state};
    std::vector<Piece> pieces;
    int64_t off = kHeader;
    for (int f = 0; f < 4; ++f) {
        if (!src[f]) continue;
        h.fields |= kFields[f].bit;
        for (int r = 0; r < kFields[f].rows; ++r) {
            char* buf = (char*)src[f] + (int64_t)r * ld * kFields[f].elem;
            pieces.push_back({off, buf, n * kFields[f].elem});
            off += n * kFields[f].elem;
        }
    }
    const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0) return ADM1_E_IO;
    bool ok = pwrite(fd, &h, sizeof(h), 0) == (ssize_t)sizeof(h) && ftruncate(fd, off) == 0 &&
              transfer(fd, pieces, true);
    ok = (close(fd) == 0) && ok;
    return ok ? ADM1_OK : ADM1_E_IO;
} catch (...) {
    return ADM1_E_IO;
}

int adm1_snapshot_info(const char* path, int64_t* n, uint32_t* fields, double* time_s)
{
    if (!path) return ADM1_E_NULL;
    const int fd = open(path, O_RDONLY);
    if (fd < 0) return ADM1_E_IO;
    Header h;
    const int rc = read_header(fd, h);
    close(fd);
    if (rc) return rc;
    if (n) *n = (int64_t)h.n;
    if (fields) *fields = h.fields;
    if (time_s) *time_s = h.time_s;
    return ADM1_OK;
}

int adm1_snapshot_read(const char* path, int64_t ld, float* pos, float* vel, float* rho,
                       double* state, int64_t* n_out)
{
    if (!path) return ADM1_E_NULL;
    const int fd = open(path, O_RDONLY);
    if (fd < 0) return ADM1_E_IO;
    Header h;
    int rc = read_header(fd, h);
    if (!rc) {
        void* const dst[4] = {pos, vel, rho, state};
        rc = read_fields(fd, h, ld, dst);
    }
    close(fd);
    if (!rc && n_out) *n_out = (int64_t)h.n;
    return rc;
}

}  // extern "C"
