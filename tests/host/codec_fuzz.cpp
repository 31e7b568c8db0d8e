// Host harness for the codec's host entry points under AddressSanitizer and
// UndefinedBehaviorSanitizer (no GPU): ct_rle_decode_host on streams written
// by a reference encoder here and on corrupted ones, ct_deflate_host and
// ct_inflate_host round trips, offsets that decrease or start below zero.
// Every buffer is exactly as large as the contract says, so an access
// outside it stops the run.
#include "../../paper_1510_00561_amd/csrc/ct_codec_api.cpp"
#include "../../paper_1510_00561_amd/csrc/ct_geometry.cpp"

#include <stdio.h>

#include <random>
#include <vector>

// The device paths are not linked: their entry points are never called here.
namespace ct {
ProfScope::ProfScope(const char* n, double by, double al, hipStream_t s) : name(n), bytes(by), alg(al), st(s) {}
void ProfScope::done() {}
namespace codec {
hipError_t launch_mc(const MCArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_rle(const RLEArgs&, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace codec
}  // namespace ct

namespace {

int failures = 0;
#define EXPECT(c)                                                  \
    do {                                                           \
        if (!(c)) {                                                \
            printf("FAILED %s at line %d\n", #c, __LINE__);       \
            ++failures;                                            \
        }                                                          \
    } while (0)

// Symbols of one plane in the documented format, from its indices.
void encode(const ct::Geometry& g, const std::vector<int16_t>& idx, int p_frame, std::vector<int16_t>& sym,
            std::vector<int32_t>& off) {
    std::vector<ct_subband> tab(g.nsub);
    ct::subband_table(g, tab.data(), g.nsub);
    sym.clear();
    off.assign(1, 0);
    for (int s = 0; s < g.nsub; ++s) {
        const ct_subband& b = tab[s];
        const bool coded = p_frame || s > 0;
        const int16_t* c = idx.data() + b.offset;
        if (!coded) {
            sym.insert(sym.end(), c, c + int64_t(b.rows) * b.cols);
        } else {
            for (int i = 0; i < b.rows; ++i) {
                int k = 0;
                while (k < b.cols) {
                    auto at = [&](int kk) { return b.transposed ? c[int64_t(kk) * b.rows + i] : c[int64_t(i) * b.cols + kk]; };
                    const int16_t v = at(k);
                    if (v != 0) {
                        sym.push_back(v);
                        ++k;
                        continue;
                    }
                    int e = k;
                    while (e < b.cols && at(e) == 0) ++e;
                    sym.push_back(0);
                    sym.push_back(int16_t(e - k));
                    k = e;
                }
            }
        }
        off.push_back(int32_t(sym.size()));
    }
}

int decode_exact(const ct_geom& geom, const std::vector<int16_t>& sym, const std::vector<int32_t>& off, int p_frame,
                 std::vector<int16_t>& out) {
    // copies into buffers of exactly the contract's sizes
    const size_t nsym = off.empty() ? 0 : size_t(off.back() > 0 ? off.back() : 0);
    std::vector<int16_t> s(sym.begin(), sym.begin() + std::min(nsym, sym.size()));
    s.resize(nsym);
    int16_t* sp = new int16_t[nsym ? nsym : 1];
    std::copy(s.begin(), s.end(), sp);
    int32_t* op = new int32_t[off.size()];
    std::copy(off.begin(), off.end(), op);
    int16_t* ip = new int16_t[out.size()];
    const int rc = ct_rle_decode_host(&geom, sp, op, p_frame, ip);
    std::copy(ip, ip + out.size(), out.begin());
    delete[] sp;
    delete[] op;
    delete[] ip;
    return rc;
}

}  // namespace

int main() {
    std::mt19937 rng(7);
    const ct_geom geoms[] = {
        {70, 90, 3, {16, 8, 4}, 0, 0}, {40, 40, 3, {8, 4, 4}, 0, 0}, {16, 16, 1, {4}, 0, 0},
        {64, 96, 2, {4, 32}, 0, 0},    {4, 4, 1, {8}, 0, 0},
    };
    int cases = 0;
    for (const ct_geom& geom : geoms) {
        ct::Geometry g;
        EXPECT(ct::resolve(&geom, &g) == CT_OK);
        for (int p_frame = 0; p_frame < 2; ++p_frame)
            for (double density : {0.0, 0.05, 0.5, 1.0}) {
                std::vector<int16_t> idx(g.ncoef);
                std::uniform_real_distribution<double> u(0, 1);
                std::uniform_int_distribution<int> val(-300, 300);
                for (auto& v : idx) v = u(rng) < density ? int16_t(val(rng)) : 0;
                std::vector<int16_t> sym;
                std::vector<int32_t> off;
                encode(g, idx, p_frame, sym, off);
                std::vector<int16_t> back(g.ncoef);
                EXPECT(decode_exact(geom, sym, off, p_frame, back) == CT_OK);
                EXPECT(back == idx);
                // DEFLATE round trips, both modes
                for (int mode = 0; mode < 2; ++mode) {
                    const int parts = mode == 0 ? g.nsub : 1;
                    std::vector<uint8_t> blob(size_t(sym.size()) * 2 * 2 + 64 * parts + 1024);
                    std::vector<uint32_t> cb(parts);
                    size_t total = 0;
                    EXPECT(ct_deflate_host(sym.data(), off.data(), g.nsub, mode, 6, blob.data(), blob.size(), cb.data(),
                                           &total) == CT_OK);
                    uint8_t* in = new uint8_t[total ? total : 1];
                    std::copy(blob.begin(), blob.begin() + total, in);
                    int16_t* out = new int16_t[sym.size() ? sym.size() : 1];
                    EXPECT(ct_inflate_host(in, cb.data(), off.data(), g.nsub, mode, out) == CT_OK);
                    EXPECT(std::equal(sym.begin(), sym.end(), out));
                    delete[] in;
                    delete[] out;
                    // a cap one byte short is a workspace error, not an overrun
                    if (total > 0) {
                        uint8_t* small = new uint8_t[total - 1 ? total - 1 : 1];
                        size_t t2 = 0;
                        const int rc = ct_deflate_host(sym.data(), off.data(), g.nsub, mode, 6, small, total - 1,
                                                       cb.data(), &t2);
                        EXPECT(rc == CT_ERR_WORKSPACE || rc == CT_OK);
                        delete[] small;
                    }
                }
                // corrupted streams: every outcome is an error code or a
                // successful parse, never an access outside the buffers
                for (int trial = 0; trial < 200; ++trial) {
                    std::vector<int16_t> bad = sym;
                    std::vector<int32_t> boff = off;
                    const int kind = trial % 5;
                    if (kind == 0 && !bad.empty()) {             // flip symbols
                        for (int f = 0; f < 3; ++f)
                            bad[rng() % bad.size()] = int16_t(int(rng() % 65536) - 32768);
                    } else if (kind == 1 && !bad.empty()) {      // truncate the stream
                        const int32_t cut = int32_t(rng() % bad.size());
                        for (auto& o : boff) o = std::min(o, cut);
                    } else if (kind == 2) {                      // a decreasing offset
                        const int s = int(rng() % g.nsub);
                        boff[s + 1] = boff[s] - 1 - int32_t(rng() % 5);
                    } else if (kind == 3) {                      // a negative start
                        boff[0] = -1 - int32_t(rng() % 5);
                    } else {                                     // shifted offsets
                        const int s = 1 + int(rng() % g.nsub);
                        boff[s] += int32_t(rng() % 7) - 3;
                        if (boff[s] < boff[s - 1]) boff[s] = boff[s - 1];
                        for (int t = s + 1; t <= g.nsub; ++t) boff[t] = std::max(boff[t], boff[s]);
                        bad.resize(size_t(std::max(boff.back(), 0)), 0);
                    }
                    std::vector<int16_t> out(g.ncoef);
                    const int rc = decode_exact(geom, bad, boff, p_frame, out);
                    EXPECT(rc == CT_OK || rc == CT_ERR_ARG);
                    if (kind == 2 || kind == 3) EXPECT(rc == CT_ERR_ARG);
                    ++cases;
                }
            }
    }
    // argument checks
    {
        const ct_geom geom{16, 16, 1, {4}, 0, 0};
        int16_t s[4] = {0};
        int32_t o[6] = {0};
        int16_t idx[512];
        EXPECT(ct_rle_decode_host(nullptr, s, o, 0, idx) == CT_ERR_ARG);
        EXPECT(ct_rle_decode_host(&geom, nullptr, o, 0, idx) == CT_ERR_ARG);
        uint32_t cb[6];
        size_t total = 0;
        EXPECT(ct_deflate_host(s, o, 0, 0, 6, nullptr, 0, cb, &total) == CT_ERR_ARG);
        EXPECT(ct_deflate_host(s, o, 5, 2, 6, nullptr, 0, cb, &total) == CT_ERR_ARG);
        EXPECT(ct_deflate_host(s, o, 5, 0, 10, nullptr, 0, cb, &total) == CT_ERR_ARG);
    }
    if (failures) return 1;
    printf("%d corrupted streams, codec host entry points clean\n", cases);
    return 0;
}
